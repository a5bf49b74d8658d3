"""Conductor-block preconditioner of the SLIM system (7).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper preconditions its GMRES solve with the constraint preconditioner of
[Qian2009] (Sec. II-C, Sec. III-E), and that definition is not given in the
paper. Reading used here: block Jacobi over conductors. Each block is the
row-equilibrated system S A restricted to one conductor's own unknowns (its RWG
edges and its triangles), and it is inverted exactly. When the system is
block-diagonal over conductors, the preconditioned operator is the identity.

A conductor with more unknowns than `cap` is cut into parts by recursive
coordinate bisection (RCB) of its triangle centroids. The rules:
  - split along the axis of largest centroid extent (lowest axis on ties);
  - order the triangles by that coordinate with a stable sort of the ascending
    triangle list;
  - the first half takes len // 2 triangles;
  - stop once a part has at most `cap` unknowns, an unknown being an owned edge
    or a triangle.
An edge belongs to the part that holds its T+ triangle. A part is grown by
max(overlap, 1) rings of edge-adjacent triangles of the same conductor.
The extended block holds the grown triangles and the edges with both
triangles among them. So no current crosses the boundary of the extended
set: each part is solved as an isolated piece of conductor. If edges with
only their T+ inside were kept, they would carry current through the cut
with no charge to balance it. At low frequency those currents are governed
by the tiny j k0 L_A term alone, and the local inverse then amplifies them
without bound. The part's rows of the inverse of the extended block are
kept (restricted additive Schwarz).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .rwg import RWG


@dataclass
class Block:
    ext: np.ndarray       # system indices (edges, then N_E + triangle), ascending within each kind
    own_pos: np.ndarray   # positions in `ext` of the unknowns this block owns
    rows: np.ndarray = None   # (len(own_pos), len(ext)) rows of the inverse, set by build()


def _edges_with_tplus_in(g: RWG, tri_set: np.ndarray) -> np.ndarray:
    """Edges whose T+ triangle is in the given set (ascending)."""
    return np.nonzero(np.isin(g.tplus, tri_set))[0]


def _unknowns(g: RWG, tris: np.ndarray) -> int:
    return int(_edges_with_tplus_in(g, tris).size + tris.size)


def rcb_parts(g: RWG, tris: np.ndarray, cap: int) -> list:
    """Recursive coordinate bisection of a triangle list into parts of at most `cap` unknowns."""
    if _unknowns(g, tris) <= cap or tris.size < 2:
        return [tris]
    c = g.centroid[tris]
    axis = int(np.argmax(c.max(axis=0) - c.min(axis=0)))
    order = tris[np.argsort(c[:, axis], kind="stable")]
    half = order.size // 2
    left, right = np.sort(order[:half]), np.sort(order[half:])
    return rcb_parts(g, left, cap) + rcb_parts(g, right, cap)


def grow(g: RWG, tris: np.ndarray, layers: int) -> np.ndarray:
    """Add `layers` rings of triangles that share an edge with the set."""
    cur = set(int(t) for t in tris)
    for _ in range(layers):
        ring = set()
        for t in cur:
            for e in g.tri_edge[t]:
                for u in (int(g.tplus[e]), int(g.tminus[e])):
                    if u not in cur:
                        ring.add(u)
        cur |= ring
    return np.array(sorted(cur), dtype=np.int64)


def _edges_inside(g: RWG, tri_set: np.ndarray) -> np.ndarray:
    """Edges with both triangles in the given set (ascending)."""
    return np.nonzero(np.isin(g.tplus, tri_set) & np.isin(g.tminus, tri_set))[0]


def partition(g: RWG, cap: int = 0, overlap: int = 2) -> list:
    """Blocks of the preconditioner; cap <= 0 keeps every conductor whole."""
    blocks = []
    for i in range(g.n_obj):
        tris = np.arange(g.obj_tri_off[i], g.obj_tri_off[i + 1])
        parts = [tris] if cap <= 0 else rcb_parts(g, tris, cap)
        for p in parts:
            ext_t = p if len(parts) == 1 else grow(g, p, max(overlap, 1))
            ext_e = _edges_inside(g, ext_t)
            own_e = _edges_with_tplus_in(g, p)
            ext = np.concatenate([ext_e, g.n_e + ext_t])
            own_pos = np.concatenate([np.searchsorted(ext_e, own_e),
                                      ext_e.size + np.searchsorted(ext_t, p)])
            blocks.append(Block(ext, own_pos))
    return blocks


def build(As: np.ndarray, blocks: list) -> list:
    """Rows of the inverse of every extended block of the equilibrated matrix As = S A."""
    for b in blocks:
        b.rows = np.linalg.inv(As[np.ix_(b.ext, b.ext)])[b.own_pos]
    return blocks


def apply(blocks: list, v: np.ndarray) -> np.ndarray:
    """z = P^{-1} v: each block writes its owned unknowns."""
    z = np.zeros_like(v)
    for b in blocks:
        z[b.ext[b.own_pos]] = b.rows @ v[b.ext]
    return z
