"""Pins of the oracle's conductor-block preconditioner and flexible GMRES.

The preconditioner is the row-equilibrated system restricted to each
conductor (or to overlapping RCB parts of a large conductor). These checks do
not use the oracle's own formula. They pin the index bookkeeping with
synthetic matrices whose preconditioned operator is exactly the identity, and
the solver against dense LU.
"""
import numpy as np
import pytest

from inputs.geometry import bar_c1, box_mesh, merge, small_boxes
from oracle import precond
from oracle.operators import Physics, dense_system
from oracle.rwg import build_rwg
from oracle.solve import fgmres, gmres, row_scaling


def _rwg(m):
    return build_rwg(m.verts, m.tris, m.obj, m.n_obj)


@pytest.fixture(scope="module")
def boxes():
    # one large box (split under a small cap) and two small ones
    parts = [box_mesh((0.0, 0.0, 0.0), (20e-6, 2e-6, 2e-6), (20, 2, 2)),
             box_mesh((25e-6, 0.0, 0.0), (4e-6, 2e-6, 2e-6), (4, 2, 2)),
             box_mesh((32e-6, 0.0, 0.0), (3e-6, 1e-6, 1e-6), (3, 1, 1))]
    return _rwg(merge(parts))


def _unknown_sets(g):
    """Conductor of every system unknown (edges, then triangles)."""
    return np.concatenate([g.edge_obj, g.obj])


@pytest.mark.parametrize("cap,overlap", [(0, 2), (120, 0), (120, 2), (60, 3)])
def test_partition_invariants(boxes, cap, overlap):
    g = boxes
    blocks = precond.partition(g, cap=cap, overlap=overlap)
    n = g.n_e + g.n_t
    owner = np.full(n, -1)
    obj_of = _unknown_sets(g)
    for k, b in enumerate(blocks):
        own = b.ext[b.own_pos]
        assert np.all(owner[own] == -1), "an unknown is owned twice"
        owner[own] = k
        # one conductor per block; edges first, then triangles, each ascending
        assert np.unique(obj_of[b.ext]).size == 1
        ne_b = np.sum(b.ext < g.n_e)
        assert np.all(np.diff(b.ext[:ne_b]) > 0) and np.all(np.diff(b.ext[ne_b:]) > 0)
        assert np.all(b.ext[ne_b:] >= g.n_e)
        # an extended edge has both triangles in the extended set: no current
        # crosses the boundary of the block
        ext_t = b.ext[ne_b:] - g.n_e
        assert np.all(np.isin(g.tplus[b.ext[:ne_b]], ext_t)) and np.all(np.isin(g.tminus[b.ext[:ne_b]], ext_t))
        # and every edge of the object with both triangles there is in the block
        inside = np.nonzero(np.isin(g.tplus, ext_t) & np.isin(g.tminus, ext_t))[0]
        assert np.array_equal(inside, b.ext[:ne_b])
        if cap > 0 and len(b.own_pos) != len(b.ext):
            assert len(b.own_pos) <= cap
    assert np.all(owner >= 0), "an unknown is owned by no block"
    # conductors within the cap stay whole
    for i in range(g.n_obj):
        ni = (g.obj_edge_off[i + 1] - g.obj_edge_off[i]) + (g.obj_tri_off[i + 1] - g.obj_tri_off[i])
        nb = len({owner[e] for e in range(g.obj_edge_off[i], g.obj_edge_off[i + 1])})
        if cap <= 0 or ni <= cap:
            assert nb == 1
        else:
            assert nb >= 2


def test_rcb_halves_and_growth(boxes):
    g = boxes
    tris = np.arange(g.obj_tri_off[0], g.obj_tri_off[1])
    parts = precond.rcb_parts(g, tris, cap=120)
    sizes = sorted(p.size for p in parts)
    # the long box is cut across its length into equal halves, recursively
    assert sum(sizes) == tris.size and sizes[-1] - sizes[0] <= 1
    assert np.array_equal(np.sort(np.concatenate(parts)), tris)
    # the first cut is along x: every triangle of the first part lies left of every one of the last
    assert g.centroid[parts[0], 0].max() <= g.centroid[parts[-1], 0].min()
    p = parts[1]
    ring = precond.grow(g, p, 1)
    added = np.setdiff1d(ring, p)
    assert added.size > 0
    # each added triangle shares an edge with the part, and every neighbour is included
    for t in added:
        nb = {int(g.tplus[e]) for e in g.tri_edge[t]} | {int(g.tminus[e]) for e in g.tri_edge[t]}
        assert nb & set(p.tolist())
    for t in p:
        for e in g.tri_edge[t]:
            assert g.tplus[e] in ring and g.tminus[e] in ring
    assert np.array_equal(precond.grow(g, p, 0), p)


def _random_blockdiag(groups, n, seed):
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n), dtype=complex)
    for idx in groups:
        k = idx.size
        B = rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k)) + 4 * np.sqrt(k) * np.eye(k)
        A[np.ix_(idx, idx)] = B
    return A


@pytest.mark.parametrize("cap,overlap", [(0, 2), (120, 0), (120, 2), (60, 3)])
def test_identity_on_matrices_block_diagonal_over_owned_sets(boxes, cap, overlap):
    """If A is block-diagonal over the owned sets, P^{-1} A = I exactly.

    This holds for whole conductors and for restricted additive Schwarz with
    any overlap: the extended block is then block-diagonal too. A wrong index
    map, a transposed block or a wrong own-row selection breaks it.
    """
    g = boxes
    blocks = precond.partition(g, cap=cap, overlap=overlap)
    n = g.n_e + g.n_t
    A = _random_blockdiag([b.ext[b.own_pos] for b in blocks], n, seed=1)
    precond.build(A, blocks)
    X = np.stack([precond.apply(blocks, A[:, j]) for j in range(n)], axis=1)
    assert np.abs(X - np.eye(n)).max() <= 1e-10


def test_overlap_differs_on_coupled_matrix(boxes):
    """With coupling across parts, a wider overlap changes the result (the extension
    is used); overlap 0 is taken as one ring, since an owned edge needs both its
    triangles in the block."""
    g = boxes
    n = g.n_e + g.n_t
    rng = np.random.default_rng(3)
    A = rng.standard_normal((n, n)) * 0.01 + np.eye(n) * 3.0
    v = rng.standard_normal(n) + 0j
    z0 = precond.apply(precond.build(A, precond.partition(g, 120, 0)), v)
    z1 = precond.apply(precond.build(A, precond.partition(g, 120, 1)), v)
    z2 = precond.apply(precond.build(A, precond.partition(g, 120, 2)), v)
    assert np.array_equal(z0, z1)
    assert np.linalg.norm(z1 - z2) > 1e-6 * np.linalg.norm(z1)


def test_fgmres_matches_lu_with_rounded_preconditioner():
    """Flexible GMRES converges with a preconditioner applied in complex64 (not linear)."""
    rng = np.random.default_rng(7)
    n = 120
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 12 * np.eye(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    Ainv = np.linalg.inv(A + 0.5 * rng.standard_normal((n, n)))
    pc = lambda v: (Ainv.astype(np.complex64) @ v.astype(np.complex64)).astype(complex)
    x, it, hist = fgmres(lambda v: A @ v, pc, b, tol=1e-12, restart=30, max_iter=300)
    ref = np.linalg.solve(A, b)
    assert hist[-1] <= 1e-12
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    # with the identity it is GMRES
    x1, it1, _ = fgmres(lambda v: A @ v, lambda v: v, b, tol=1e-10, restart=30, max_iter=300)
    x2, it2, _ = gmres(lambda v: A @ v, b, tol=1e-10, restart=30, max_iter=300)
    assert it1 == it2 and np.linalg.norm(x1 - x2) <= 1e-12 * np.linalg.norm(x2)


@pytest.mark.slow
def test_single_conductor_block_is_the_system():
    """One conductor, no cap: P = S A, so one flexible-GMRES step solves it."""
    m = bar_c1(div=(8, 1, 1), length=20e-6)
    g = _rwg(m)
    S = dense_system(g, Physics(10e9))
    A = S.dense()
    s = row_scaling(g.n_e, g.n_t, g.length.mean())
    As = s[:, None] * A
    blocks = precond.build(As, precond.partition(g))
    assert len(blocks) == 1
    rng = np.random.default_rng(0)
    b = rng.standard_normal(As.shape[0]) + 1j * rng.standard_normal(As.shape[0])
    x, it, hist = fgmres(lambda v: As @ v, lambda v: precond.apply(blocks, v), b, tol=1e-10, restart=20, max_iter=20)
    assert it <= 2 and hist[-1] <= 1e-10


@pytest.mark.slow
def test_conductor_blocks_solve_multi_object_system():
    """Three copper boxes at 10 GHz: preconditioned FGMRES reaches 1e-8 in a few
    iterations and agrees with dense LU, while unpreconditioned GMRES is slower."""
    m = small_boxes(3, seed=2)
    g = _rwg(m)
    S = dense_system(g, Physics(10e9))
    A = S.dense()
    s = row_scaling(g.n_e, g.n_t, g.length.mean())
    As = s[:, None] * A
    rng = np.random.default_rng(1)
    b = rng.standard_normal(As.shape[0]) + 1j * rng.standard_normal(As.shape[0])
    ref = np.linalg.solve(As, b)
    blocks = precond.build(As, precond.partition(g))
    x, it, hist = fgmres(lambda v: As @ v, lambda v: precond.apply(blocks, v), b, tol=1e-8, restart=50, max_iter=200)
    assert hist[-1] <= 1e-8 and it <= 25
    assert np.linalg.norm(x - ref) <= 1e-5 * np.linalg.norm(ref)
    _, it0, hist0 = gmres(lambda v: As @ v, b, tol=1e-8, restart=50, max_iter=4 * it)
    assert hist0[-1] > 1e-8
