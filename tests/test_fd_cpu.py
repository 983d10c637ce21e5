"""The finite-difference machinery of the gradient tests, checked on the CPU.

The worker of ``tests/fd_chain.py`` (central differences of the oracle's chain
forward) must reproduce dense binary64 autograd of the expanded chain on a
shrunk chain (bond 4), along seeded directions and at single entries; this pins
both the worker and the oracle's chain against torch's autograd.
"""
import numpy as np
import torch

import oracle as O
from tests import fd_chain


def test_central_differences_match_dense_autograd_on_a_shrunk_chain():
    fd_chain.init(threads=2, bond=4)
    wl, syms, host = fd_chain._STATE["wl"], fd_chain._STATE["syms"], fd_chain._STATE["host"]
    dense = {k: torch.from_numpy(O.expand(host[k], syms[k])).requires_grad_(k in ("E", "A", "W")) for k in host}
    cur = dict(dense)
    for st in wl.steps:
        cur[st.w] = torch.einsum(st.einsum, cur[st.u], cur[st.v])
    (cur[wl.output] * dense["R"]).sum().backward()
    rng = np.random.default_rng(3)
    for k in ("E", "A", "W"):
        grad, zero_ok = O.reduce_full(dense[k].grad.numpy(), syms[k])
        assert zero_ok
        jobs = [(k, "dir", 7 + j, 1e-6) for j in range(2)]
        jobs += [(k, "entry", int(e), 1.0) for e in rng.choice(host[k].size, 4, replace=False)]
        for job in jobs:
            fd = fd_chain.central_difference(job)
            an = float(np.sum(grad * fd_chain.direction(host[k].shape, job[1], job[2])))
            scale = abs(fd) if job[1] == "dir" else float(np.max(np.abs(grad)))
            assert abs(fd - an) <= 1e-8 * scale, (job, fd, an)
