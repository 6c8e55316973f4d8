"""Pins of the oracle's blocked DOF numbering (oracle_map_blocked): the skeleton
DOFs (global node (I,J,K) with a coordinate that is a multiple of N) first, in
the lexicographic order of the global nodes, then every element's (N-1)^3
interior DOFs, element after element.

The numbering is a relabelling of the lexicographic one, so it is pinned
against that (already pinned) numbering and against the closed forms of the
box, not against itself:
- the relabelling is one permutation P of the DOFs, the same for every local
  copy of a node;
- the block sizes have closed forms: S skeleton DOFs, E (N-1)^3 interior ones;
- the skeleton labels keep the lexicographic order, the interior labels are
  the stated contiguous ranges, and an interior DOF appears in exactly one
  element;
- the operator is P A P^T exactly (the oracle sums a DOF's element
  contributions in element order under either numbering, so the results are
  bit-identical), and CG on P b follows the same residual history.
"""
import numpy as np
import pytest

import inputs
from oracle import MASS_INVDEG, Mesh


def perm(lex, blk):
    """The relabelling lexicographic DOF -> blocked DOF, checked to be one
    well-defined permutation (every local copy of a DOF agrees)."""
    keep = lex.map >= 0
    assert np.array_equal(keep, blk.map >= 0)
    P = np.full(lex.NG, -1, dtype=np.int64)
    P[lex.map[keep]] = blk.map[keep]
    assert np.array_equal(P[lex.map[keep]], blk.map[keep]), "two copies of one node got different labels"
    assert np.array_equal(np.sort(P), np.arange(lex.NG)), "not a permutation of the DOFs"
    return P


def skeleton_count(nx, ny, nz, N, dirichlet):
    """Skeleton DOFs of the box by inclusion of whole planes and lines: the
    nodes with at least one coordinate on an element boundary."""
    k = 1 if dirichlet else 0
    L = [n * N + 1 - 2 * k for n in (nx, ny, nz)]
    # skeleton coordinates along an axis: element boundaries 0..n (minus the two box faces when masked)
    s = [n + 1 - 2 * k for n in (nx, ny, nz)]
    free = [Ld - sd for Ld, sd in zip(L, s)]  # coordinates strictly inside an element
    return L[0] * L[1] * L[2] - free[0] * free[1] * free[2]


BOXES = [(1, 1, 1, 1), (2, 2, 2, 1), (1, 1, 1, 2), (2, 3, 2, 2), (3, 2, 2, 3), (2, 2, 3, 4), (1, 2, 1, 5),
         (2, 1, 2, 7), (1, 1, 2, 9), (2, 1, 1, 15)]


@pytest.mark.parametrize("dirichlet", [False, True])
@pytest.mark.parametrize("nx,ny,nz,N", BOXES)
def test_blocked_is_a_relabelling_with_the_stated_blocks(nx, ny, nz, N, dirichlet):
    if dirichlet and min(nx, ny, nz) * N < 2:
        pytest.skip("a Dirichlet box needs interior nodes")
    lex = Mesh(nx, ny, nz, N, dirichlet=dirichlet)
    blk = Mesh(nx, ny, nz, N, dirichlet=dirichlet, blocked=True)
    assert blk.NG == lex.NG
    E, ni = nx * ny * nz, (N - 1) ** 3
    S = skeleton_count(nx, ny, nz, N, dirichlet)
    assert blk.NS == S and S + E * ni == blk.NG
    P = perm(lex, blk)
    # global coordinates of every lexicographic DOF
    k = 1 if dirichlet else 0
    gx, gy = nx * N + 1 - 2 * k, ny * N + 1 - 2 * k
    g = np.arange(lex.NG)
    I, J, K = g % gx + k, (g // gx) % gy + k, g // (gx * gy) + k
    on_skel = (I % N == 0) | (J % N == 0) | (K % N == 0)
    # skeleton DOFs get the labels 0..S-1 in lexicographic order
    assert np.array_equal(P[on_skel], np.arange(S))
    # interior DOFs: element e's local node (a,b,c) -> S + e (N-1)^3 + (a-1) + (N-1)((b-1) + (N-1)(c-1))
    m = blk.map.reshape(E, N + 1, N + 1, N + 1)  # [e][c][b][a]
    if N >= 2:
        inner = m[:, 1:N, 1:N, 1:N].reshape(E, ni)
        want = S + np.arange(E)[:, None] * ni + np.arange(ni)[None, :]
        assert np.array_equal(inner, want)
        # and no interior DOF is seen by any other local node
        count = np.bincount(blk.map[blk.map >= 0], minlength=blk.NG)
        assert np.all(count[S:] == 1)
    # every skeleton DOF is on a face, edge or vertex of each element that sees it
    a = np.arange(N + 1)
    edge = (a == 0) | (a == N)
    face = edge[None, None, :] | edge[None, :, None] | edge[:, None, None]
    assert np.all((m < S)[:, face] | (m < 0)[:, face])


@pytest.mark.parametrize("dirichlet", [False, True])
@pytest.mark.parametrize("nx,ny,nz,N,jitter", [(3, 2, 2, 3, 0.1), (2, 2, 2, 5, 0.05), (2, 1, 2, 7, 0.0),
                                               (2, 2, 1, 2, 0.1), (1, 2, 2, 11, 0.05)])
def test_blocked_operator_is_the_permuted_operator(nx, ny, nz, N, jitter, dirichlet):
    lex = Mesh(nx, ny, nz, N, jitter=jitter, seed=3, dirichlet=dirichlet)
    blk = Mesh(nx, ny, nz, N, jitter=jitter, seed=3, dirichlet=dirichlet, blocked=True)
    P = perm(lex, blk)
    x = inputs.random_vector(lex.NG, 11)
    xb = np.empty_like(x)
    xb[P] = x
    y = lex.ax(x, 0.9)
    yb = blk.ax(xb, 0.9)
    assert np.array_equal(yb[P], y)  # bit-identical: same sums in the same order
    assert np.array_equal(blk.diag(0.9)[P], lex.diag(0.9))


def test_blocked_invdeg_mass_and_cg_history():
    lex = Mesh(3, 2, 2, 4, jitter=0.1, seed=8, mass=MASS_INVDEG)
    blk = Mesh(3, 2, 2, 4, jitter=0.1, seed=8, mass=MASS_INVDEG, blocked=True)
    P = perm(lex, blk)
    assert np.array_equal(blk.geo, lex.geo)  # geometry is per local node, untouched by the numbering
    b = inputs.random_vector(lex.NG, 5)
    bb = np.empty_like(b)
    bb[P] = b
    r = lex.cg(b, 1.0, fixed_iters=40)
    rb = blk.cg(bb, 1.0, fixed_iters=40)
    # the dot products sum in another order: equal to rounding
    assert np.allclose(rb["res"], r["res"], rtol=1e-11, atol=0)
    assert np.allclose(rb["x"][P], r["x"], rtol=0, atol=1e-10 * np.abs(r["x"]).max())
