"""The allocation-free entry point hlbm_set_porosity_noalloc against
hlbm_set_porosity: the same porosity field (bitwise) and the same flow after
it, on two calls in a row on two lattices (the second smaller), a rejected
field followed by an accepted one (the flag is cleared by each call), and no
device memory added to the lattice."""
import ctypes as C

import numpy as np
import pytest

from tests.pairs import Spec, make_gpu, say

pytestmark = pytest.mark.gpu


def H():
    from paper_2606_31707_amd import hlbm
    return hlbm


def _field(n, seed):
    return np.random.default_rng(seed).uniform(0.0, 1.0, n)


def test_noalloc_matches_set_porosity():
    import torch
    h = H()
    say("no-alloc porosity")
    for (nx, ny), seed in (((150, 41), 1), ((67, 19), 2)):  # the second call smaller
        s = Spec(nx=nx, ny=ny, tau=0.6, u_in=0.05, cyl=None)
        A, B = make_gpu(s), make_gpu(s)
        d = _field(s.n, seed)
        A.set_porosity(d)
        held = B.device_bytes()
        dt = torch.tensor(d, device="cuda")
        st = B._lib.hlbm_set_porosity_noalloc(B._h, C.c_void_p(dt.data_ptr()), s.n)
        assert st == h.OK, h.load_library().hlbm_last_error()
        assert B.device_bytes() == held
        assert np.array_equal(A.porosity(), B.porosity())
        for G in (A, B):
            G.init_equilibrium()
            G.run_primal(50)
        assert np.array_equal(A.populations(), B.populations())
        # a rejected field, then an accepted one on the same lattice
        bad = dt.clone()
        bad[s.n // 2] = 1.5
        st = B._lib.hlbm_set_porosity_noalloc(B._h, C.c_void_p(bad.data_ptr()), s.n)
        assert st == h.E_INVALID
        st = B._lib.hlbm_set_porosity_noalloc(B._h, C.c_void_p(dt.data_ptr()), s.n)
        assert st == h.OK
        assert np.array_equal(A.porosity(), B.porosity())
        with pytest.raises(h.HlbmError):
            B.set_porosity_noalloc(dt[:-1].contiguous())
        A.close()
        B.close()
