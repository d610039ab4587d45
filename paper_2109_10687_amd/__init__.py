"""MI355X (gfx950) Clover-Wilson quark solver: Dirac apply, SAP preconditioner,
BiCGStab and mixed-precision defect correction (arXiv 2109.10687), as a C-ABI
HIP library (libddsolve.so, include/ddsolve.h) with a thin ctypes binding;
batched right-hand sides on the matrix cores, and the derivative of
|D^{-1} phi|^2 with respect to the links (autograd.py)."""
from .binding import (DD_BATCH_INNER_PLAIN, DD_BATCH_INNER_SAP, DD_DEBUG_ZERO_OMEGA_F16, DD_DEBUG_ZERO_OMEGA_F32, DD_F16, DD_F32, DD_F64, DD_KT_BLAS, DD_KT_DIRAC_F16,
                      DD_KT_DIRAC_F16IN, DD_KT_DIRAC_F32, DD_KT_DIRAC_F64, DD_KT_DIRAC_MRHS, DD_KT_DIRAC_MULTI, DD_KT_FORCE, DD_KT_SAP,
                      DD_OP_A, DD_OP_D, DD_OP_DDAG, DD_SOLVE_F32_SAP, DD_SOLVE_F64_PLAIN, DD_SOLVE_MIXED,
                      DD_SOLVE_MIXED_GCR, DD_SOLVE_FGMRES, EXPORTS, KERNEL_CLASSES, DDError, Multi, Params, Solver, bicgstab_solve,
                      bicgstab_solve_batch, bicgstab_solve_dagger, dd_batch_set_variant, dd_batch_tuning,
                      dd_batch_variant_name, dd_create, dd_destroy, dd_field_bytes, dd_force, dd_load_gauge,
                      dd_pack_spinor, dd_set_csw, dd_spinor_norm2, dd_timing_enable, dd_timing_query,
                      dd_unpack_spinor, dirac_apply, dirac_apply_batch, dirac_apply_packed, dirac_apply_packed_f16in, lib,
                      sap_precondition)
