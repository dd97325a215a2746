"""fracture_set_allocator: the library's device memory from PyTorch's caching allocator.

A Newton loop run with every block taken from torch gives bitwise the same state as the
library's own pool; torch accounts for the blocks while the objects live and gets them back
when they are destroyed; objects made under one allocator outlive a change of allocator.
"""
import gc

import numpy as np
import pytest
import torch

from paper_1806_09924_amd import binding as B
from gpu_util import Problem, host

pytestmark = pytest.mark.gpu


def _newton(P):
    u, phi, po, pt = P.dstate()
    st = B.newton(P.mesh, P.prm, u, phi, po, pt)
    return st, host(u), host(phi)


def test_torch_allocator_same_results_and_accounting():
    torch.cuda.synchronize()
    ref_st, ref_u, ref_phi = _newton(Problem(2, 2.0, 128))
    try:
        B.set_allocator("torch")
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        P = Problem(2, 2.0, 128)                 # mesh, system, hierarchy, Krylov bases from torch
        st, u, phi = _newton(P)
        held = torch.cuda.memory_allocated() - base
        assert held > 8 * P.mesh.n_solve * 8     # at least the system vectors and a few Krylov vectors
        assert st["status"] == B.FR_OK
        assert st["iterations"] == ref_st["iterations"] and st["linear_iters"] == ref_st["linear_iters"]
        assert np.array_equal(u, ref_u) and np.array_equal(phi, ref_phi)
        # an object made under torch's allocator outlives the switch back to the pool
        B.set_allocator(None)
        st2, u2, phi2 = _newton(P)
        assert np.array_equal(u2, ref_u) and np.array_equal(phi2, ref_phi)
        del P
        gc.collect()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() - base <= held // 100
    finally:
        B.set_allocator(None)
