"""Seeded synthetic inputs shared by the CPU oracle and the GPU library tests.

Nothing here computes any part of the contraction method: this package maps
(seed, tensor id, element index) to values (``philox``), describes the
workloads' shapes and symmetry labels (``configs``), and — in
``synth/csrc/synth_gen.hip`` — fills device buffers with the very same values
for the GPU side.
"""
from .philox import DIST_NORMAL, DIST_UNIFORM, fill, philox4x32_10, values_at  # noqa: F401
from . import configs  # noqa: F401


def host_input(wl, name: str):
    """The standard reduced form of input ``name`` of workload ``wl``, binary64, on the host
    (through the C twin of the generator when it is built: the same bits, faster)."""
    from . import host
    op = wl.operands[name]
    if host.available():
        return host.fill(wl.reduced_shape(name), wl.seed, op.tensor_id, op.dist, op.scale)
    return fill(wl.reduced_shape(name), wl.seed, op.tensor_id, op.dist, op.scale)
