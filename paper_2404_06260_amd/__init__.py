"""MI355X library for the localized model-order-reduction finite element method.

The compute path is the HIP library ``libmor.so`` (``csrc/``, C-ABI in ``include/mor.h``);
``mor`` is its ctypes binding.  Importing ``mor`` raises if the library is not built.
"""
