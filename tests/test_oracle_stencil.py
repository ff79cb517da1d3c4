"""Pins of the oracle's velocity sets and equilibrium (Sec. 2.1).

The D2Q9/D3Q19 sets must reproduce the lattice isotropy identities up to
fourth order with c_s^2 = 1/3, and the second-order equilibrium must carry
exactly the moments rho, rho v and rho/3 I + rho v v.
"""
import itertools

import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("kind", [O.D2Q9, O.D3Q19])
def test_isotropy(kind):
    c, w, opp = O.stencil(kind)
    dim = 2 if kind == O.D2Q9 else 3
    c = c[:, :dim].astype(float)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs(w @ c).max() < 1e-16
    assert np.abs(np.einsum("i,ia,ib->ab", w, c, c) - np.eye(dim) / 3).max() < 1e-16
    assert np.abs(np.einsum("i,ia,ib,ic->abc", w, c, c, c)).max() < 1e-16
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    I = np.eye(dim)
    ref = (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I)
           + np.einsum("ad,bc->abcd", I, I)) / 9.0
    assert np.abs(m4 - ref).max() < 1e-16
    # opposite directions
    assert np.array_equal(c[opp], -c)
    # every velocity appears once
    assert len({tuple(v) for v in c}) == len(c)


@pytest.mark.parametrize("kind", [O.D2Q9, O.D3Q19])
def test_equilibrium_moments(kind):
    c, w, _ = O.stencil(kind)
    dim = 2 if kind == O.D2Q9 else 3
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = rng.uniform(0.8, 1.2)
        v = np.zeros(3)
        v[:dim] = rng.uniform(-0.1, 0.1, dim)
        feq = O.equilibrium(kind, rho, v)
        cc = c.astype(float)
        assert abs(feq.sum() - rho) < 1e-15
        assert np.abs(feq @ cc - rho * v).max() < 1e-15
        P = np.einsum("i,ia,ib->ab", feq, cc, cc)[:dim, :dim]
        ref = rho / 3 * np.eye(dim) + rho * np.outer(v[:dim], v[:dim])
        assert np.abs(P - ref).max() < 1e-15


@pytest.mark.parametrize("kind", [O.D2Q9, O.D3Q19])
def test_equilibrium_at_rest_is_weights(kind):
    _, w, _ = O.stencil(kind)
    assert np.array_equal(O.equilibrium(kind, 1.0, [0, 0, 0]), w)


def test_d2q9_table_values():
    """Hand-written D2Q9 table: the canonical direction order is part of the
    exchange format, so it is pinned literally."""
    c, w, opp = O.stencil(O.D2Q9)
    assert [tuple(v[:2]) for v in c] == [(0, 0), (1, 0), (0, 1), (1, 1), (-1, 1),
                                         (-1, 0), (0, -1), (-1, -1), (1, -1)]
    assert np.allclose(w, [4 / 9] + [1 / 9, 1 / 9, 1 / 36, 1 / 36] * 2, rtol=0, atol=1e-17)
    assert list(opp) == [0, 5, 6, 7, 8, 1, 2, 3, 4]


def test_d3q19_table_values():
    c, w, opp = O.stencil(O.D3Q19)
    axes = [v for v in c if np.abs(v).sum() == 1]
    edges = [v for v in c if np.abs(v).sum() == 2]
    assert len(axes) == 6 and len(edges) == 12
    assert all(abs(w[i] - 1 / 18) < 1e-17 for i in range(19) if np.abs(c[i]).sum() == 1)
    assert all(abs(w[i] - 1 / 36) < 1e-17 for i in range(19) if np.abs(c[i]).sum() == 2)
    assert list(opp[1:10]) == list(range(10, 19))
