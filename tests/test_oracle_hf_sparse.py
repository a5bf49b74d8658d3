"""Oracle pins of the high-frequency sparse interior operators (Sec. III-A, point 3):
the full-radius limit is the dense operator of eq. (4)-(6), the dropped interactions are
negligible once the skin depth is small (and not at low frequency), and the truncation
error falls with the radius."""
import numpy as np
import pytest

from inputs.geometry import merge, random_complex, split_ring_mesh
from oracle.hf_sparse import interacting, object_pairs, sparse_interior_blocks, sparse_LK, z_pattern
from oracle.operators import Physics, interior_blocks, interior_LK
from oracle.rwg import build_rwg, matrix_Ix_and_gram

UM = 1e-6


@pytest.fixture(scope="module")
def ring():
    """One copper split ring (radius 20 um, width 4, thickness 1, gap 4), coarse: 156 triangles."""
    m = merge([split_ring_mesh((0.0, 0.0, 0.0), 20 * UM, 4 * UM, 1 * UM, 4 * UM, 19)])
    return build_rwg(m.verts, m.tris, m.obj, m.n_obj)


@pytest.fixture(scope="module")
def dense_100ghz(ring):
    return interior_blocks(ring, Physics(100e9))


def test_full_radius_is_the_dense_operator(ring, dense_100ghz):
    """With r beyond the object's extent every triangle pair interacts: Z~_t, M~ and Y_eq
    are the dense Z, M = Y_eq Z and Y_eq bit for bit."""
    ext = np.ptp(ring.verts, axis=0).max()
    inner, P = sparse_interior_blocks(ring, Physics(100e9), 2.0 * ext)
    assert P[0].all()
    assert np.array_equal(inner.Z[0], dense_100ghz.Z[0])
    assert np.array_equal(inner.M[0], dense_100ghz.M[0])
    assert np.array_equal(inner.Yeq[0], dense_100ghz.Yeq[0])


def test_pattern_symmetric_local_and_defined_by_pairs(ring):
    """The pattern holds the diagonal, is symmetric, and (m, n) is in it exactly when an
    interacting triangle pair couples an edge of one triangle to an edge of the other."""
    r = 3.0 * ring.diam.max()
    P = z_pattern(ring, 0, r)
    assert np.all(np.diag(P)) and np.array_equal(P, P.T)
    assert 0.05 < P.mean() < 0.8
    T, U = object_pairs(ring, 0)
    close = interacting(ring, T, U, r)
    Q = np.zeros_like(P)
    for t, u in zip(T[close], U[close]):
        for m in ring.tri_edge[t]:
            for n in ring.tri_edge[u]:
                Q[m, n] = Q[n, m] = True
    assert np.array_equal(P, Q)
    # brute force on a few entries off the pattern: no pair of their triangles is within r
    far = np.argwhere(~P)[:20]
    for m, n in far:
        for t in (ring.tplus[m], ring.tminus[m]):
            for u in (ring.tplus[n], ring.tminus[n]):
                assert np.linalg.norm(ring.centroid[t] - ring.centroid[u]) > r


def test_distant_interactions_negligible_at_high_frequency(ring, dense_100ghz):
    """100 GHz (skin depth 0.21 um against 5-10 um triangles): dropping the triangle pairs
    more than two triangle diameters apart leaves Z~ = L~^{-1}(K~ + I_x/2) c equal to Z to
    rounding, because the conductor kernel has decayed by e^{-2 diam / delta}."""
    ph = Physics(100e9)
    r = 2.0 * ring.diam.max()
    Ix, _ = matrix_Ix_and_gram(ring)
    Lc, Kc = sparse_LK(ring, 0, ph.kc, r)
    Z = (-1.0 / (1j * ph.omega * ph.eps_c)) * np.linalg.solve(Lc, Kc + 0.5 * Ix)
    Zd = dense_100ghz.Z[0]
    assert np.linalg.norm(Z - Zd) / np.linalg.norm(Zd) < 1e-12
    # the dropped entries of L_kc themselves are below rounding relative to its largest entry
    Ld, _ = interior_LK(ring, 0, ph.kc)
    assert np.abs(Ld - Lc).max() < 1e-15 * np.abs(Ld).max()


def test_truncation_error_falls_with_radius(ring, dense_100ghz):
    """The product e = Z~_t H against the dense e = Z H: the relative error falls with r
    and is below 1e-5 at four triangle diameters."""
    ph = Physics(100e9)
    H = random_complex(ring.n_e, 3)
    e = dense_100ghz.Z[0] @ H
    Ix, _ = matrix_Ix_and_gram(ring)
    errs = []
    for f in (1.5, 2.5, 4.0):
        r = f * ring.diam.max()
        Lc, Kc = sparse_LK(ring, 0, ph.kc, r)
        Zt = np.where(z_pattern(ring, 0, r), (-1.0 / (1j * ph.omega * ph.eps_c)) * np.linalg.solve(Lc, Kc + 0.5 * Ix), 0)
        errs.append(np.linalg.norm(Zt @ H - e) / np.linalg.norm(e))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-5


def test_low_frequency_is_not_local(ring):
    """At 100 MHz (skin depth 6.6 um, about the object's cross-section) the interior kernel
    has not decayed over the same radius: the variant is for developed skin effect only."""
    ph = Physics(100e6)
    r = 2.0 * ring.diam.max()
    Ix, _ = matrix_Ix_and_gram(ring)
    Lc, Kc = sparse_LK(ring, 0, ph.kc, r)
    Ld, Kd = interior_LK(ring, 0, ph.kc)
    assert np.linalg.norm(Ld - Lc) / np.linalg.norm(Ld) > 1e-3
