"""MI355X-native irreducible-representation-alignment contraction of tensors with
cyclic-group (Z_G) or product-of-cyclic-group symmetry.

The compute path is the HIP library ``libsymtensor.so`` (C ABI in
include/symtensor.h); this package marshals torch tensors into it.
"""
from .symtensor import (  # noqa: F401
    SymTensor, align, contract_into, derived_charges, derived_sectors, einsum, group_size, output_like,
    plan, read_timing, sector_gemm, sector_gemm_workspace_size, set_timing, unalign,
)
