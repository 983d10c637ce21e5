"""CPU FP64 reference for cyclic-group-symmetric tensor contraction.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are its only users.  The GPU library never imports, links or
calls it, and it shares no code with the GPU library.

Pins (each checked by the CPU test suite against something other than the
oracle's own formulas): brute force on tiny inputs, agreement of the five
forms, the conservation invariant of the output, G = 1 against numpy.einsum,
the block-diagonal matrix product, the Z_2 x Z_3 = Z_6 isomorphism, the
closed-form flop counts of the paper, bfloat16 rounding against torch, charge
tables by relabelling, U(1) and complex tensors against np.einsum, and
subgroup modes against the smaller cyclic group and brute force.
"""
from .symcontract import (  # noqa: F401
    Group, Sym, allowed, implicit_sector, full_sectors, stored_tuples, expand, reduce_full, lookup,
    parse_einsum, contracted_sign_ratio, output_symmetry, same_symmetry, check_operands,
    flop_count, contract_dense, contract_blocks, sample_contract, sample_contract_allowed, reduced_value_fn,
    contract_bruteforce, kron_delta, alignment_deltas, align_u, align_v, unalign_w,
    contract_irrep_aligned, aligned_shape, bf16_round, bf16_split,
)
