// Host-side decomposition: index sets, CSR patterns, element colouring, neighbour pairs.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace mor {

// SpMM tiles of the block CG: runs of whole row aggregates of at most kHaloRows rows and
// halo_nnz_cap(cap) padded CSR entries whose II columns (the tile's halo: every row of P the tile reads)
// number at most cap, so that one 256-byte column slice of every halo row and the tile's
// CSR fit in LDS.
constexpr int kHaloRows = 64;
constexpr int kHaloCap = 176;   // the largest halo; a context may choose a smaller one (kHaloCaps)
constexpr int kHaloCaps[5] = {48, 64, 96, 128, 176};
// two-level preconditioner: a coarse block is a run of this many consecutive row aggregates
constexpr int kCoarseAgg = 8;
// padded CSR entries per tile for a halo cap (a Kuhn-cube row has 15 II entries, padded to 16)
constexpr int halo_nnz_cap(int cap) { return cap * 8 < 1024 ? cap * 8 : 1024; }

struct HostMesh {
  int64_t n_nodes = 0, n_tets = 0;
  std::vector<double> xyz;
  std::vector<int32_t> tets;
  std::vector<uint8_t> dirichlet;
  std::vector<int32_t> star;    // tets per node
  std::vector<uint8_t> colour;  // greedy element colouring: tets sharing a node differ
  int ncolours = 0;
  // Kuhn lattice: when every node sits near a point of a regular grid (spacing estimated from
  // the axis-aligned edges) and every edge joins two grid points whose offset lies in
  // {0,1}^3 or {0,-1}^3, lat holds each node's integer grid coordinates (3 per node)
  bool lattice = false;
  std::vector<int32_t> lat;
};

// The 15-point stencil of a Kuhn lattice: slot 0 the node itself, slots 1..7 the forward
// offsets, slots 8..14 their negatives; slot 15 pads a row to 16 entries.
constexpr int kStencil = 16;
constexpr int kKuhnOff[15][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1},
                                 {1, 1, 1}, {-1, 0, 0}, {0, -1, 0}, {0, 0, -1}, {-1, -1, 0}, {-1, 0, -1},
                                 {0, -1, -1}, {-1, -1, -1}};

// Local numbering of one subdomain: [P | V\P | I\V | B], each part sorted by global id.
struct HostSub {
  int nP = 0, nV = 0, nI = 0, nB = 0, nL = 0;
  std::vector<int32_t> nodes;              // global ids, nL
  std::vector<int32_t> rp, col, ii_end;    // CSR of the omega_i^+ matrices over the local nodes
  std::vector<int32_t> rpV, colV;          // CSR of K_i over V_i (local ids < nV)
  std::vector<int32_t> ltet;               // 4 local ids per local tet (-1 = Dirichlet), colour-sorted
  std::vector<int32_t> tetg;               // global tet id per local tet
  std::vector<uint8_t> core;               // 1 if the local tet lies in omega_i
  std::vector<int32_t> colour_ptr;         // local tets of colour c: [colour_ptr[c], colour_ptr[c+1])
  std::vector<int32_t> bp;                 // aggregates of I rows: block b = rows [bp[b], bp[b+1]), size <= 8
  std::vector<int32_t> bpL;                // aggregates of all nL rows: bp, then the B rows in runs of 8
  std::vector<int32_t> htile;              // SpMM tiles, 4 ints each: first row, rows, first halo entry, halo size
  std::vector<int32_t> halo;               // each tile's halo rows (local ids < nI), ascending
  std::vector<int32_t> hrowp;              // per I row (+1): start of its padded II entries in hpe / hpp
  std::vector<int32_t> hpe;                // padded II entries: CSR entry id, or -1 (weight 0)
  std::vector<uint16_t> hpp;               // padded II entries: the column's position in the tile halo
  std::vector<uint16_t> hself;             // per I row: the row's own position in its tile halo
  std::vector<int32_t> rcb;                // per I row: its coarse block (aggregate / kCoarseAgg)
  std::vector<int32_t> rcbL;               // per local row: its coarse block over the aggregates bpL
  // Box form of the interior (on a Kuhn lattice, when I is a full box of grid points):
  // extents nx, ny, nz; smap[(z*ny + y)*nx + x] = local row of the grid point (x, y, z) of the
  // box; spos[16 r + s] = CSR entry of row r's stencil slot s in the II block, or -1.
  int bx = 0, by = 0, bz = 0;
  std::vector<int32_t> smap, spos;
};

// omega_0: the elements in two or more subdomains, with A_0's pattern over their free nodes.
struct HostOmega0 {
  HostSub sub;                 // nodes = free nodes of omega_0 tets (all in the "I" part), rp/col, ltet
  // neighbour pairs (i < j) with triplets (row in P_i, row in P_j, A_0 slot)
  std::vector<int32_t> pair_i, pair_j, pair_first, pair_count;
  std::vector<int32_t> trip;   // 3 per triplet
};

int build_mesh(HostMesh& m, std::string& err);
int build_sub(const HostMesh& m, const int32_t* ext, const uint8_t* in_core, int64_t n_ext, HostSub& s,
              std::string& err, int halo_cap = kHaloCap);
// owner / position of every free node in its P_i; error unless the P_i partition the free nodes
int build_owner(const HostMesh& m, const std::vector<HostSub>& subs, std::vector<int32_t>& owner,
                std::vector<int32_t>& ownpos, std::string& err);
int build_omega0(const HostMesh& m, const std::vector<HostSub>& subs, const int64_t* ext_ptr, const int32_t* ext,
                 const uint8_t* in_core, const std::vector<int32_t>& owner, const std::vector<int32_t>& ownpos,
                 HostOmega0& o, std::string& err);

}  // namespace mor
