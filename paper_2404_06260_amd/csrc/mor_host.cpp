// Host-side decomposition for the local reduction (integer work, negligible next to the solves).
//
// Index sets follow Sections 3-4 of the paper: I = free nodes interior to omega_i^+, B = free
// nodes on the boundary of omega_i^+, V_i = free nodes of omega_i, P_i = the interior of omega_i
// (where the stitching operator of Definition 3.1 keeps values).  A free node is interior to a
// union of tets exactly when every tet around it belongs to the union, which is how both are
// decided here.  omega_0 and the neighbour pairs follow Section 6, step 3.
#include "mor_host.h"

#include <algorithm>
#include <cmath>
#include <climits>
#include <cstring>
#include <numeric>

namespace mor {

static double tet_det(const HostMesh& m, int64_t t) {
  const int32_t* v = &m.tets[4 * t];
  const double* x0 = &m.xyz[3 * (int64_t)v[0]];
  double e[3][3];
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 3; ++d) e[a][d] = m.xyz[3 * (int64_t)v[a + 1] + d] - x0[d];
  return e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) - e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
         e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
}

// Kuhn-lattice detection.  The grid spacing per axis: a first guess h0 is the median of each
// edge's largest coordinate difference; edge components above h0 / 2 are then single grid steps
// (plus noise from node jitter), whose median estimates the spacing, which is finally rounded so
// that the node extent along the axis is a whole number of steps.  Each node takes the nearest
// grid point.  The structure is then verified, not assumed: every tet edge must join grid points
// whose offset is a Kuhn offset and no two nodes may share a grid point.  Any failure leaves
// m.lattice false.
static void detect_lattice(HostMesh& m) {
  m.lattice = false;
  m.lat.clear();
  if (m.n_nodes < 8) return;
  static const int E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  const int64_t stride = std::max<int64_t>(1, m.n_tets / 200000);
  auto edge_diff = [&](int64_t t, const int* ed, double* d) {
    const double* a = &m.xyz[3 * (int64_t)m.tets[4 * t + ed[0]]];
    const double* b = &m.xyz[3 * (int64_t)m.tets[4 * t + ed[1]]];
    for (int ax = 0; ax < 3; ++ax) d[ax] = std::fabs(b[ax] - a[ax]);
  };
  std::vector<double> big;
  for (int64_t t = 0; t < m.n_tets; t += stride)
    for (const auto& ed : E) {
      double d[3];
      edge_diff(t, ed, d);
      big.push_back(std::max(d[0], std::max(d[1], d[2])));
    }
  if (big.size() < 16) return;
  std::nth_element(big.begin(), big.begin() + big.size() / 2, big.end());
  const double h0 = big[big.size() / 2];
  if (!(h0 > 0.0)) return;
  std::vector<double> len[3];
  for (int64_t t = 0; t < m.n_tets; t += stride)
    for (const auto& ed : E) {
      double d[3];
      edge_diff(t, ed, d);
      for (int ax = 0; ax < 3; ++ax)
        if (d[ax] > 0.5 * h0) len[ax].push_back(d[ax]);
    }
  double h[3], lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t v = 0; v < m.n_nodes; ++v)
    for (int ax = 0; ax < 3; ++ax) {
      lo[ax] = std::min(lo[ax], m.xyz[3 * v + ax]);
      hi[ax] = std::max(hi[ax], m.xyz[3 * v + ax]);
    }
  for (int ax = 0; ax < 3; ++ax) {
    if (len[ax].size() < 16) return;
    std::nth_element(len[ax].begin(), len[ax].begin() + len[ax].size() / 2, len[ax].end());
    const double he = len[ax][len[ax].size() / 2];
    const double steps = std::nearbyint((hi[ax] - lo[ax]) / he);
    if (!(he > 0.0) || !(steps >= 1.0)) return;
    h[ax] = (hi[ax] - lo[ax]) / steps;
  }
  std::vector<int32_t> lat(3 * m.n_nodes);
  for (int64_t v = 0; v < m.n_nodes; ++v)
    for (int ax = 0; ax < 3; ++ax) {
      const double q = std::nearbyint((m.xyz[3 * v + ax] - lo[ax]) / h[ax]);
      if (!(q >= 0.0 && q < 2097152.0)) return;   // 21 bits per axis for the uniqueness key
      lat[3 * v + ax] = (int32_t)q;
    }
  for (int64_t t = 0; t < m.n_tets; ++t)
    for (const auto& ed : E) {
      const int32_t* a = &lat[3 * (int64_t)m.tets[4 * t + ed[0]]];
      const int32_t* b = &lat[3 * (int64_t)m.tets[4 * t + ed[1]]];
      int pos = 0, neg = 0;
      for (int ax = 0; ax < 3; ++ax) {
        const int d = b[ax] - a[ax];
        if (d < -1 || d > 1) return;
        pos += d > 0;
        neg += d < 0;
      }
      if ((pos > 0) == (neg > 0)) return;   // zero, or a mixed-sign offset
    }
  std::vector<uint64_t> key(m.n_nodes);
  for (int64_t v = 0; v < m.n_nodes; ++v)
    key[v] = ((uint64_t)lat[3 * v] << 42) | ((uint64_t)lat[3 * v + 1] << 21) | (uint64_t)lat[3 * v + 2];
  std::sort(key.begin(), key.end());
  if (std::adjacent_find(key.begin(), key.end()) != key.end()) return;
  m.lat.swap(lat);
  m.lattice = true;
}

// Box form of a subdomain's interior on a Kuhn lattice (see HostSub): empty unless the I rows
// fill a box of grid points and every II entry is a stencil slot.
static void build_box(const HostMesh& m, HostSub& s) {
  s.bx = s.by = s.bz = 0;
  s.smap.clear();
  s.spos.clear();
  if (!m.lattice || s.nI == 0) return;
  int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {-1, -1, -1};
  for (int r = 0; r < s.nI; ++r)
    for (int ax = 0; ax < 3; ++ax) {
      const int q = m.lat[3 * (int64_t)s.nodes[r] + ax];
      lo[ax] = std::min(lo[ax], q);
      hi[ax] = std::max(hi[ax], q);
    }
  const int64_t ext[3] = {hi[0] - lo[0] + 1, hi[1] - lo[1] + 1, hi[2] - lo[2] + 1};
  if (ext[0] * ext[1] * ext[2] != (int64_t)s.nI) return;
  std::vector<int32_t> smap(s.nI, -1);
  auto cell = [&](int r, int* q) {
    for (int ax = 0; ax < 3; ++ax) q[ax] = m.lat[3 * (int64_t)s.nodes[r] + ax] - lo[ax];
  };
  for (int r = 0; r < s.nI; ++r) {
    int q[3];
    cell(r, q);
    int32_t& slot = smap[((int64_t)q[2] * ext[1] + q[1]) * ext[0] + q[0]];
    if (slot >= 0) return;
    slot = r;
  }
  std::vector<int32_t> spos((size_t)kStencil * s.nI, -1);
  for (int r = 0; r < s.nI; ++r) {
    int q[3];
    cell(r, q);
    for (int e = s.rp[r]; e < s.ii_end[r]; ++e) {
      int w[3];
      cell(s.col[e], w);
      int k = -1;
      for (int sl = 0; sl < 15 && k < 0; ++sl)
        if (w[0] - q[0] == kKuhnOff[sl][0] && w[1] - q[1] == kKuhnOff[sl][1] && w[2] - q[2] == kKuhnOff[sl][2]) k = sl;
      if (k < 0 || spos[(size_t)kStencil * r + k] >= 0) return;
      spos[(size_t)kStencil * r + k] = e;
    }
  }
  s.bx = (int)ext[0];
  s.by = (int)ext[1];
  s.bz = (int)ext[2];
  s.smap.swap(smap);
  s.spos.swap(spos);
}

int build_mesh(HostMesh& m, std::string& err) {
  m.star.assign(m.n_nodes, 0);
  for (int64_t t = 0; t < m.n_tets; ++t) {
    for (int a = 0; a < 4; ++a) {
      const int32_t v = m.tets[4 * t + a];
      if (v < 0 || v >= m.n_nodes) {
        err = "tet " + std::to_string(t) + " references node " + std::to_string(v) + " out of range";
        return -1;
      }
      m.star[v]++;
    }
    const double det = tet_det(m, t);
    if (!(det > 0.0)) {
      err = "tet " + std::to_string(t) + " has non-positive volume (det J = " + std::to_string(det) + ")";
      return -1;
    }
  }
  std::vector<uint64_t> used(m.n_nodes, 0);
  m.colour.assign(m.n_tets, 0);
  int nc = 0;
  for (int64_t t = 0; t < m.n_tets; ++t) {
    uint64_t u = 0;
    for (int a = 0; a < 4; ++a) u |= used[m.tets[4 * t + a]];
    if (u == ~0ull) {
      err = "element colouring needs more than 64 colours";
      return -1;
    }
    const int c = __builtin_ctzll(~u);
    m.colour[t] = (uint8_t)c;
    nc = std::max(nc, c + 1);
    for (int a = 0; a < 4; ++a) used[m.tets[4 * t + a]] |= (1ull << c);
  }
  m.ncolours = nc;
  detect_lattice(m);
  return 0;
}

// CSR pattern over local ids from a list of local tets (4 ids, -1 skipped); rows [0, nrows)
static void tet_pattern(const std::vector<int32_t>& ltet, const std::vector<uint8_t>* mask, int nrows,
                        std::vector<int32_t>& rp, std::vector<int32_t>& col) {
  const int64_t nt = (int64_t)ltet.size() / 4;
  std::vector<int32_t> cnt(nrows + 1, 0);
  for (int64_t t = 0; t < nt; ++t) {
    if (mask && !(*mask)[t]) continue;
    for (int a = 0; a < 4; ++a) {
      const int r = ltet[4 * t + a];
      if (r >= 0 && r < nrows) cnt[r + 1]++;
    }
  }
  for (int r = 0; r < nrows; ++r) cnt[r + 1] += cnt[r];
  std::vector<int32_t> adj(cnt[nrows]);
  std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t t = 0; t < nt; ++t) {
    if (mask && !(*mask)[t]) continue;
    for (int a = 0; a < 4; ++a) {
      const int r = ltet[4 * t + a];
      if (r >= 0 && r < nrows) adj[fill[r]++] = (int32_t)t;
    }
  }
  rp.assign(nrows + 1, 0);
  col.clear();
  std::vector<int32_t> buf;
  for (int r = 0; r < nrows; ++r) {
    buf.clear();
    for (int k = cnt[r]; k < cnt[r + 1]; ++k) {
      const int64_t t = adj[k];
      for (int b = 0; b < 4; ++b) {
        const int c = ltet[4 * t + b];
        if (c >= 0) buf.push_back(c);
      }
    }
    std::sort(buf.begin(), buf.end());
    buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
    col.insert(col.end(), buf.begin(), buf.end());
    rp[r + 1] = (int32_t)col.size();
  }
}

static void colour_sort(const HostMesh& m, HostSub& s, std::vector<int32_t>& ltet, std::vector<int32_t>& tetg,
                        std::vector<uint8_t>& core) {
  const int64_t nt = (int64_t)tetg.size();
  std::vector<int32_t> cnt(m.ncolours + 1, 0);
  for (int64_t t = 0; t < nt; ++t) cnt[m.colour[tetg[t]] + 1]++;
  for (int c = 0; c < m.ncolours; ++c) cnt[c + 1] += cnt[c];
  s.colour_ptr = cnt;
  std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
  s.ltet.assign(4 * nt, -1);
  s.tetg.assign(nt, 0);
  s.core.assign(nt, 0);
  for (int64_t t = 0; t < nt; ++t) {
    const int64_t d = fill[m.colour[tetg[t]]]++;
    for (int a = 0; a < 4; ++a) s.ltet[4 * d + a] = ltet[4 * t + a];
    s.tetg[d] = tetg[t];
    s.core[d] = core.empty() ? 0 : core[t];
  }
}

// Greedy SpMM tiling over whole aggregates, in row order: a tile grows while it has at most
// kHaloRows rows and halo_nnz_cap(cap) padded entries and its halo (the union of the II columns of its
// rows) at most kHaloCap rows.  Each row's II entries are padded to a multiple of 8 (entry -1,
// weight 0) so the kernel takes them in chunks of 8 without bounds tests.
static int padded_ii(const HostSub& s, int r) { return (s.ii_end[r] - s.rp[r] + 7) / 8 * 8; }

static int build_halo_tiles(HostSub& s, int cap, std::string& err) {
  s.htile.clear();
  s.halo.clear();
  s.hpe.clear();
  s.hpp.clear();
  s.hrowp.assign(s.nI + 1, 0);
  s.hself.assign(s.nI, 0);
  std::vector<int32_t> stamp(s.nI, -1), cur, add;
  const int nb = (int)s.bp.size() - 1;
  int b = 0;
  while (b < nb) {
    const int tid = (int)s.htile.size() / 4;
    const int row0 = s.bp[b];
    cur.clear();
    int b1 = b, npad = 0;
    while (b1 < nb) {
      const int r0 = s.bp[b1], r1 = s.bp[b1 + 1];
      int addpad = 0;
      for (int r = r0; r < r1; ++r) addpad += padded_ii(s, r);
      if (b1 > b && (r1 - row0 > kHaloRows || npad + addpad > halo_nnz_cap(cap))) break;
      add.clear();
      for (int r = r0; r < r1; ++r)
        for (int e = s.rp[r]; e < s.ii_end[r]; ++e) {
          const int cc = s.col[e];
          if (stamp[cc] != tid) {
            stamp[cc] = tid;
            add.push_back(cc);
          }
        }
      if (b1 > b && (int)(cur.size() + add.size()) > cap) {
        for (int cc : add) stamp[cc] = -1;
        break;
      }
      cur.insert(cur.end(), add.begin(), add.end());
      npad += addpad;
      ++b1;
    }
    std::sort(cur.begin(), cur.end());
    const int row1 = s.bp[b1];
    s.htile.push_back(row0);
    s.htile.push_back(row1 - row0);
    s.htile.push_back((int32_t)s.halo.size());
    s.htile.push_back((int32_t)cur.size());
    auto pos = [&](int cc) { return (int)(std::lower_bound(cur.begin(), cur.end(), cc) - cur.begin()); };
    for (int r = row0; r < row1; ++r) {
      s.hrowp[r] = (int32_t)s.hpe.size();
      const int pad = padded_ii(s, r);
      for (int k = 0; k < pad; ++k) {
        const int e = s.rp[r] + k;
        const bool real = e < s.ii_end[r];
        s.hpe.push_back(real ? e : -1);
        s.hpp.push_back((uint16_t)(real ? pos(s.col[e]) : 0));
      }
      s.hself[r] = (uint16_t)pos(r);
    }
    s.halo.insert(s.halo.end(), cur.begin(), cur.end());
    b = b1;
  }
  s.hrowp[s.nI] = (int32_t)s.hpe.size();
  // the SpMM kernel indexes LDS with these: check every bound it relies on
  int next = 0;
  for (size_t t = 0; t < s.htile.size(); t += 4) {
    const int r0 = s.htile[t], nr = s.htile[t + 1], h0 = s.htile[t + 2], nh = s.htile[t + 3];
    if (r0 != next || nr < 1 || nr > kHaloRows || nh < 1 || nh > cap || cap > kHaloCap || h0 + nh > (int)s.halo.size() ||
        s.hrowp[r0 + nr] - s.hrowp[r0] > halo_nnz_cap(cap)) {
      err = "internal: SpMM tile out of bounds";
      return -1;
    }
    next = r0 + nr;
    for (int r = r0; r < r0 + nr; ++r) {
      if (s.hself[r] >= nh || s.halo[h0 + s.hself[r]] != r || (s.hrowp[r + 1] - s.hrowp[r]) % 8 != 0) {
        err = "internal: SpMM tile misses its own row";
        return -1;
      }
      int real = 0;
      for (int k = s.hrowp[r]; k < s.hrowp[r + 1]; ++k) {
        const int e = s.hpe[k];
        if (s.hpp[k] >= nh || (e >= 0 && (e < s.rp[r] || e >= s.ii_end[r] || s.halo[h0 + s.hpp[k]] != s.col[e]))) {
          err = "internal: SpMM tile halo misses a column";
          return -1;
        }
        real += e >= 0;
      }
      if (real != s.ii_end[r] - s.rp[r]) {
        err = "internal: SpMM tile drops an entry";
        return -1;
      }
    }
  }
  if (next != s.nI) {
    err = "internal: SpMM tiles do not cover the interior rows";
    return -1;
  }
  return 0;
}

int build_sub(const HostMesh& m, const int32_t* ext, const uint8_t* in_core, int64_t n_ext, HostSub& s,
              std::string& err, int halo_cap) {
  std::vector<int32_t> starE(m.n_nodes, 0), starC(m.n_nodes, 0);
  std::vector<int32_t> touched;
  touched.reserve(n_ext);
  for (int64_t k = 0; k < n_ext; ++k) {
    const int32_t t = ext[k];
    if (t < 0 || t >= m.n_tets) {
      err = "subdomain tet id out of range";
      return -1;
    }
    for (int a = 0; a < 4; ++a) {
      const int32_t v = m.tets[4 * (int64_t)t + a];
      if (starE[v] == 0) touched.push_back(v);
      starE[v]++;
      if (in_core[k]) starC[v]++;
    }
  }
  std::sort(touched.begin(), touched.end());
  std::vector<int32_t> P, VmP, ImV, B;
  for (int32_t v : touched) {
    if (m.dirichlet[v]) continue;
    const bool interior = starE[v] == m.star[v];
    const bool in_v = starC[v] > 0;
    if (in_v && !interior) {
      err = "omega_i touches the boundary of omega_i^+ (the extension must be at least one layer)";
      return -1;
    }
    if (!interior) B.push_back(v);
    else if (!in_v) ImV.push_back(v);
    else if (starC[v] == m.star[v]) P.push_back(v);
    else VmP.push_back(v);
  }
  s.nP = (int)P.size();
  s.nV = s.nP + (int)VmP.size();
  s.nI = s.nV + (int)ImV.size();
  s.nB = (int)B.size();
  s.nL = s.nI + s.nB;
  if (s.nI == 0 || s.nB == 0) {
    err = "subdomain without interior or interface degrees of freedom";
    return -1;
  }
  s.nodes.clear();
  s.nodes.reserve(s.nL);
  for (auto* part : {&P, &VmP, &ImV, &B}) s.nodes.insert(s.nodes.end(), part->begin(), part->end());
  std::vector<int32_t>& lid = starE;   // reuse as global -> local map
  std::vector<int32_t> ltet(4 * n_ext), tetg(n_ext);
  std::vector<uint8_t> core(n_ext);
  auto local_tets = [&]() {
    for (int32_t v : touched) lid[v] = -1;
    for (int i = 0; i < s.nL; ++i) lid[s.nodes[i]] = i;
    for (int64_t k = 0; k < n_ext; ++k) {
      const int32_t t = ext[k];
      tetg[k] = t;
      core[k] = in_core[k] ? 1 : 0;
      for (int a = 0; a < 4; ++a) {
        const int32_t v = m.tets[4 * (int64_t)t + a];
        ltet[4 * k + a] = m.dirichlet[v] ? -1 : lid[v];
      }
    }
    colour_sort(m, s, ltet, tetg, core);
    tet_pattern(s.ltet, nullptr, s.nL, s.rp, s.col);
  };
  local_tets();
  // Aggregates of at most 8 I rows for the block-Jacobi preconditioner of the CG: in id
  // order, an unaggregated row takes its unaggregated higher-numbered neighbours of the same
  // group (P, V\P, I\V).  On a Kuhn cube these are the 7 forward corners of a 2x2x2 cell
  // block.  A row joins only while the aggregate's halo (the I rows its rows couple to) stays
  // within the LDS tile capacity, so every aggregate fits one SpMM tile on any mesh (on a Kuhn
  // mesh the halo is at most 65 rows).  Rows are then renumbered aggregate by aggregate, the aggregates of each group in
  // Morton (Z-curve) order of their first node, so that runs of consecutive aggregates (the
  // SpMM tiles) are compact bricks rather than strips.
  {
    const int gb[4] = {0, s.nP, s.nV, s.nI};
    std::vector<int32_t> agg(s.nI, -1), order, hstamp(s.nI, -1);
    auto halo_add = [&](int v, int tag, bool commit) {   // I columns of row v new to aggregate `tag`
      int k = 0;
      for (int e = s.rp[v]; e < s.rp[v + 1]; ++e) {
        const int cc = s.col[e];
        if (cc < s.nI && hstamp[cc] != tag) {
          ++k;
          if (commit) hstamp[cc] = tag;
        }
      }
      return k;
    };
    std::vector<int32_t> bp{0};
    int gfirst[4] = {0, 0, 0, 0};   // first aggregate of each group
    order.reserve(s.nI);
    for (int g = 0; g < 3; ++g) {
      gfirst[g] = (int)bp.size() - 1;
      for (int v = gb[g]; v < gb[g + 1]; ++v) {
        if (agg[v] >= 0) continue;
        const int b = (int)bp.size() - 1;
        agg[v] = b;
        order.push_back(v);
        int n = 1;
        int hsize = halo_add(v, b, true);
        if (hsize > halo_cap) {
          err = "a row couples to " + std::to_string(hsize) + " interior rows, more than the SpMM halo capacity " +
                std::to_string(halo_cap) + " (choose a larger spmm_rows, up to 176)";
          return -1;
        }
        for (int e = s.rp[v]; e < s.rp[v + 1] && n < 8; ++e) {
          const int u = s.col[e];
          if (u > v && u < gb[g + 1] && agg[u] < 0) {
            const int k = halo_add(u, b, false);
            if (hsize + k > halo_cap) continue;
            hsize += halo_add(u, b, true);
            agg[u] = b;
            order.push_back(u);
            ++n;
          }
        }
        bp.push_back((int32_t)order.size());
      }
    }
    gfirst[3] = (int)bp.size() - 1;
    {
      double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
      for (int i = 0; i < s.nI; ++i)
        for (int a = 0; a < 3; ++a) {
          const double x = m.xyz[3 * (int64_t)s.nodes[i] + a];
          lo[a] = std::min(lo[a], x);
          hi[a] = std::max(hi[a], x);
        }
      auto morton = [&](int node) {
        uint64_t key = 0;
        uint32_t qv[3];
        for (int a = 0; a < 3; ++a) {
          const double w = hi[a] > lo[a] ? (m.xyz[3 * (int64_t)node + a] - lo[a]) / (hi[a] - lo[a]) : 0.0;
          qv[a] = (uint32_t)std::min(1023.0, std::max(0.0, w * 1023.0 + 0.5));
        }
        for (int bit = 9; bit >= 0; --bit)
          for (int a = 0; a < 3; ++a) key = (key << 1) | ((qv[a] >> bit) & 1u);
        return key;
      };
      const int na = (int)bp.size() - 1;
      std::vector<uint64_t> key(na);
      for (int b = 0; b < na; ++b) key[b] = morton(s.nodes[order[bp[b]]]);
      std::vector<int32_t> ord2, bp2{0};
      ord2.reserve(s.nI);
      for (int g = 0; g < 3; ++g) {
        std::vector<int32_t> ids(gfirst[g + 1] - gfirst[g]);
        std::iota(ids.begin(), ids.end(), gfirst[g]);
        std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) { return key[a] < key[b]; });
        for (int b : ids) {
          for (int k = bp[b]; k < bp[b + 1]; ++k) ord2.push_back(order[k]);
          bp2.push_back((int32_t)ord2.size());
        }
      }
      order.swap(ord2);
      bp.swap(bp2);
    }
    std::vector<int32_t> nodes2(s.nL);
    for (int i = 0; i < s.nI; ++i) nodes2[i] = s.nodes[order[i]];
    for (int i = s.nI; i < s.nL; ++i) nodes2[i] = s.nodes[i];
    s.nodes.swap(nodes2);
    s.bp.swap(bp);
    local_tets();
  }
  s.bpL = s.bp;
  for (int r = s.nI; r < s.nL; r += 8) s.bpL.push_back(std::min(r + 8, s.nL));
  s.rcb.assign(s.nI, 0);
  for (int b = 0; b + 1 < (int)s.bp.size(); ++b)
    for (int r = s.bp[b]; r < s.bp[b + 1]; ++r) s.rcb[r] = b / kCoarseAgg;
  s.rcbL.assign(s.nL, 0);
  for (int b = 0; b + 1 < (int)s.bpL.size(); ++b)
    for (int r = s.bpL[b]; r < s.bpL[b + 1]; ++r) s.rcbL[r] = b / kCoarseAgg;
  s.ii_end.resize(s.nI);
  for (int r = 0; r < s.nI; ++r) {
    const int32_t* b = s.col.data() + s.rp[r];
    const int32_t* e = s.col.data() + s.rp[r + 1];
    s.ii_end[r] = (int32_t)(std::lower_bound(b, e, s.nI) - s.col.data());
  }
  if (build_halo_tiles(s, halo_cap, err)) return -1;
  build_box(m, s);
  tet_pattern(s.ltet, &s.core, s.nV, s.rpV, s.colV);
  for (int32_t c : s.colV)
    if (c >= s.nV) {
      err = "internal: K_i pattern leaves V_i";
      return -1;
    }
  return 0;
}

int build_owner(const HostMesh& m, const std::vector<HostSub>& subs, std::vector<int32_t>& owner,
                std::vector<int32_t>& ownpos, std::string& err) {
  owner.assign(m.n_nodes, -1);
  ownpos.assign(m.n_nodes, -1);
  for (size_t i = 0; i < subs.size(); ++i) {
    const HostSub& s = subs[i];
    for (int p = 0; p < s.nP; ++p) {
      const int32_t v = s.nodes[p];
      if (owner[v] >= 0) {
        err = "node " + std::to_string(v) + " is interior to two subdomains: cores must overlap in one layer";
        return -1;
      }
      owner[v] = (int32_t)i;
      ownpos[v] = p;
    }
  }
  for (int64_t v = 0; v < m.n_nodes; ++v)
    if (!m.dirichlet[v] && owner[v] < 0) {
      err = "free node " + std::to_string(v) + " is interior to no subdomain";
      return -1;
    }
  return 0;
}

int build_omega0(const HostMesh& m, const std::vector<HostSub>& subs, const int64_t* ext_ptr, const int32_t* ext,
                 const uint8_t* in_core, const std::vector<int32_t>& owner, const std::vector<int32_t>& ownpos,
                 HostOmega0& o, std::string& err) {
  (void)err;
  std::vector<uint8_t> cnt(m.n_tets, 0);
  for (size_t i = 0; i < subs.size(); ++i)
    for (int64_t k = ext_ptr[i]; k < ext_ptr[i + 1]; ++k)
      if (in_core[k] && cnt[ext[k]] < 255) cnt[ext[k]]++;
  std::vector<int32_t> t0;
  for (int64_t t = 0; t < m.n_tets; ++t)
    if (cnt[t] >= 2) t0.push_back((int32_t)t);
  std::vector<int32_t> lid(m.n_nodes, -1);
  std::vector<int32_t> nodes;
  for (int32_t t : t0)
    for (int a = 0; a < 4; ++a) {
      const int32_t v = m.tets[4 * (int64_t)t + a];
      if (!m.dirichlet[v] && lid[v] < 0) {
        lid[v] = 0;
        nodes.push_back(v);
      }
    }
  std::sort(nodes.begin(), nodes.end());
  for (size_t i = 0; i < nodes.size(); ++i) lid[nodes[i]] = (int32_t)i;
  HostSub& s = o.sub;
  s.nodes = nodes;
  s.nP = s.nV = 0;
  s.nI = s.nL = (int)nodes.size();
  s.nB = 0;
  std::vector<int32_t> ltet(4 * t0.size()), tetg(t0);
  std::vector<uint8_t> core;
  for (size_t k = 0; k < t0.size(); ++k)
    for (int a = 0; a < 4; ++a) {
      const int32_t v = m.tets[4 * (int64_t)t0[k] + a];
      ltet[4 * k + a] = m.dirichlet[v] ? -1 : lid[v];
    }
  colour_sort(m, s, ltet, tetg, core);
  tet_pattern(s.ltet, nullptr, s.nL, s.rp, s.col);
  // neighbour pairs: A_0 entries coupling P_i and P_j (i < j)
  struct Trip { int64_t key; int32_t p, q, slot; };
  std::vector<Trip> tr;
  const int64_t nsub = (int64_t)subs.size();
  for (int r = 0; r < s.nL; ++r) {
    const int32_t gp = nodes[r];
    const int32_t i = owner[gp];
    for (int e = s.rp[r]; e < s.rp[r + 1]; ++e) {
      const int32_t gq = nodes[s.col[e]];
      const int32_t j = owner[gq];
      if (i < j) tr.push_back({(int64_t)i * nsub + j, ownpos[gp], ownpos[gq], e});
    }
  }
  std::stable_sort(tr.begin(), tr.end(), [](const Trip& a, const Trip& b) { return a.key < b.key; });
  o.pair_i.clear(); o.pair_j.clear(); o.pair_first.clear(); o.pair_count.clear();
  o.trip.resize(3 * tr.size());
  for (size_t k = 0; k < tr.size(); ++k) {
    if (k == 0 || tr[k].key != tr[k - 1].key) {
      o.pair_i.push_back((int32_t)(tr[k].key / nsub));
      o.pair_j.push_back((int32_t)(tr[k].key % nsub));
      o.pair_first.push_back((int32_t)k);
      o.pair_count.push_back(0);
    }
    o.pair_count.back()++;
    o.trip[3 * k] = tr[k].p;
    o.trip[3 * k + 1] = tr[k].q;
    o.trip[3 * k + 2] = tr[k].slot;
  }
  return 0;
}

}  // namespace mor
