"""Seeded synthetic inputs: closed conductor surface meshes and excitation vectors.

This module is shared by the FP64 oracle and by the GPU library's tests and
benchmark.  It holds no arithmetic of the solver itself: it only places
vertices, connects them into outward-oriented triangles and draws random
numbers.  Everything the method computes (basis functions, operators, grids)
is done separately on each side.

All lengths are in metres.  A mesh is a triple

    verts : float64 (n_vert, 3)
    tris  : int32   (n_tri, 3)   counter-clockwise seen from outside
    obj   : int32   (n_tri,)     object id of every triangle, non-decreasing

Workloads (sizes follow the paper's structures: copper conductors of very
uneven size, split-ring metasurface cells, interconnect bundles):

    bar_c1()            one 100 x 2 x 2 um bar, 592 triangles / 888 edges
    srr_array_c2()      8 x 8 split rings, 300 triangles each
    line_bundle_c3()    200 lines, log-uniform lengths 10-500 um
    conductors_c5()     2000 boxes and plates, Pareto-tailed triangle counts
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

UM = 1e-6


@dataclass
class Mesh:
    verts: np.ndarray
    tris: np.ndarray
    obj: np.ndarray
    n_obj: int
    info: dict = field(default_factory=dict)

    @property
    def n_tri(self) -> int:
        return int(self.tris.shape[0])


def _orient(tri_list, verts, outward):
    """Flip triangles whose right-hand normal disagrees with `outward`."""
    out = []
    for (a, b, c), n in zip(tri_list, outward):
        e = np.cross(verts[b] - verts[a], verts[c] - verts[a])
        out.append((a, b, c) if float(np.dot(e, n)) > 0.0 else (a, c, b))
    return out


def box_mesh(origin, size, div):
    """Closed box surface, every face a structured grid split into triangles.

    origin, size: 3-vectors (metres); div: (nx, ny, nz) >= 1.
    Returns (verts, tris) with 4*(nx*ny + ny*nz + nz*nx) triangles.
    """
    nx, ny, nz = (int(d) for d in div)
    ox, oy, oz = (float(o) for o in origin)
    lx, ly, lz = (float(s) for s in size)
    vid = {}
    verts = []

    def v(i, j, k):
        key = (i, j, k)
        if key not in vid:
            vid[key] = len(verts)
            verts.append((ox + lx * i / nx, oy + ly * j / ny, oz + lz * k / nz))
        return vid[key]

    quads, normals = [], []
    # faces x = 0 / x = nx
    for i, s in ((0, -1.0), (nx, 1.0)):
        for j in range(ny):
            for k in range(nz):
                quads.append((v(i, j, k), v(i, j + 1, k), v(i, j + 1, k + 1), v(i, j, k + 1)))
                normals.append((s, 0.0, 0.0))
    for j, s in ((0, -1.0), (ny, 1.0)):
        for i in range(nx):
            for k in range(nz):
                quads.append((v(i, j, k), v(i + 1, j, k), v(i + 1, j, k + 1), v(i, j, k + 1)))
                normals.append((0.0, s, 0.0))
    for k, s in ((0, -1.0), (nz, 1.0)):
        for i in range(nx):
            for j in range(ny):
                quads.append((v(i, j, k), v(i + 1, j, k), v(i + 1, j + 1, k), v(i, j + 1, k)))
                normals.append((0.0, 0.0, s))
    verts = np.asarray(verts, dtype=np.float64)
    tl, nl = [], []
    for (a, b, c, d), n in zip(quads, normals):
        tl += [(a, b, c), (a, c, d)]
        nl += [n, n]
    tris = np.asarray(_orient(tl, verts, np.asarray(nl)), dtype=np.int32)
    return verts, tris


def split_ring_mesh(center, r_mid, width, thick, gap, n_theta):
    """Closed split-ring (annular sector extruded in z), 8*n_theta + 4 triangles."""
    cx, cy, cz = (float(c) for c in center)
    rin, rout = r_mid - width / 2.0, r_mid + width / 2.0
    th_gap = gap / r_mid
    th0, th1 = th_gap / 2.0, 2.0 * math.pi - th_gap / 2.0
    verts = []
    # vertex (station s, corner c) c: 0=(rin,z0) 1=(rout,z0) 2=(rout,z1) 3=(rin,z1)
    for s in range(n_theta + 1):
        th = th0 + (th1 - th0) * s / n_theta
        ct, st = math.cos(th), math.sin(th)
        for r, z in ((rin, 0.0), (rout, 0.0), (rout, thick), (rin, thick)):
            verts.append((cx + r * ct, cy + r * st, cz + z))
    verts = np.asarray(verts, dtype=np.float64)

    def vi(s, c):
        return 4 * s + c

    tl, nl = [], []
    for s in range(n_theta):
        thm = th0 + (th1 - th0) * (s + 0.5) / n_theta
        rh = np.array([math.cos(thm), math.sin(thm), 0.0])
        faces = (((0, 1), (0.0, 0.0, -1.0)),   # bottom
                 ((1, 2), tuple(rh)),          # outer wall
                 ((2, 3), (0.0, 0.0, 1.0)),    # top
                 ((3, 0), tuple(-rh)))         # inner wall
        for (c0, c1), n in faces:
            a, b, c, d = vi(s, c0), vi(s, c1), vi(s + 1, c1), vi(s + 1, c0)
            tl += [(a, b, c), (a, c, d)]
            nl += [n, n]
    for s, sign, th in ((0, -1.0, th0), (n_theta, 1.0, th1)):
        tang = np.array([-math.sin(th), math.cos(th), 0.0]) * sign
        a, b, c, d = vi(s, 0), vi(s, 1), vi(s, 2), vi(s, 3)
        tl += [(a, b, c), (a, c, d)]
        nl += [tuple(tang), tuple(tang)]
    tris = np.asarray(_orient(tl, verts, np.asarray(nl)), dtype=np.int32)
    return verts, tris


def ring_mesh(center, r_mid, width, thick, n_theta):
    """Closed ring of rectangular section (a split ring without its gap): a genus-1
    surface of 8*n_theta triangles.  Station s sits at angle 2 pi s / n_theta; its four
    section corners are (r_in, z0), (r_out, z0), (r_out, z1), (r_in, z1)."""
    cx, cy, cz = (float(c) for c in center)
    rin, rout = r_mid - width / 2.0, r_mid + width / 2.0
    verts = []
    for s in range(n_theta):
        th = 2.0 * math.pi * s / n_theta
        ct, st = math.cos(th), math.sin(th)
        for r, z in ((rin, 0.0), (rout, 0.0), (rout, thick), (rin, thick)):
            verts.append((cx + r * ct, cy + r * st, cz + z))
    verts = np.asarray(verts, dtype=np.float64)
    tl, nl = [], []
    for s in range(n_theta):
        s1 = (s + 1) % n_theta
        thm = 2.0 * math.pi * (s + 0.5) / n_theta
        rh = np.array([math.cos(thm), math.sin(thm), 0.0])
        for (c0, c1), n in (((0, 1), (0.0, 0.0, -1.0)), ((1, 2), tuple(rh)), ((2, 3), (0.0, 0.0, 1.0)),
                            ((3, 0), tuple(-rh))):
            a, b, c, d = 4 * s + c0, 4 * s + c1, 4 * s1 + c1, 4 * s1 + c0
            tl += [(a, b, c), (a, c, d)]
            nl += [n, n]
    tris = np.asarray(_orient(tl, verts, np.asarray(nl)), dtype=np.int32)
    return verts, tris


def merge(parts):
    """Concatenate (verts, tris) parts into one Mesh; part k becomes object k."""
    vs, ts, os_ = [], [], []
    off = 0
    for k, (v, t) in enumerate(parts):
        vs.append(v)
        ts.append(t + off)
        os_.append(np.full(t.shape[0], k, dtype=np.int32))
        off += v.shape[0]
    return Mesh(np.concatenate(vs), np.concatenate(ts).astype(np.int32),
                np.concatenate(os_), len(parts))


def box_divisions(size, n_tri_target):
    """Grid divisions of a box whose surface gets about n_tri_target triangles."""
    lx, ly, lz = size
    area = 2.0 * (lx * ly + ly * lz + lz * lx)
    a = math.sqrt(2.0 * area / n_tri_target)
    return tuple(max(1, int(round(s / a))) for s in size)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def bar_c1(div=(36, 2, 2), length=100 * UM, side=2 * UM):
    """Copper bar 100 x 2 x 2 um, 36 x 2 x 2 quads per face direction."""
    v, t = box_mesh((0.0, -side / 2, -side / 2), (length, side, side), div)
    m = merge([(v, t)])
    m.info = dict(workload="bar", length=length, side=side, div=tuple(div))
    return m


def small_boxes(n=3, seed=0, tri_range=(20, 80)):
    """A few small boxes of uneven size: a tiny multi-object case for parity."""
    rng = np.random.default_rng(seed)
    parts = []
    x = 0.0
    for _ in range(n):
        w, h = rng.uniform(1.0, 3.0, size=2) * UM
        l = rng.uniform(3.0, 12.0) * UM
        t = int(rng.integers(tri_range[0], tri_range[1] + 1))
        div = box_divisions((l, w, h), t)
        parts.append(box_mesh((x, rng.uniform(-2, 2) * UM, rng.uniform(-2, 2) * UM), (l, w, h), div))
        x += l + 3.0 * UM
    m = merge(parts)
    m.info = dict(workload="small_boxes", seed=seed)
    return m


def srr_array_c2(nx=8, ny=8, pitch=60 * UM, r_mid=20 * UM, width=4 * UM,
                 thick=1 * UM, gap=4 * UM, n_theta=37):
    """nx x ny split-ring cells (8*n_theta+4 = 300 triangles per ring)."""
    parts = []
    for j in range(ny):
        for i in range(nx):
            parts.append(split_ring_mesh((i * pitch, j * pitch, 0.0), r_mid, width, thick, gap, n_theta))
    m = merge(parts)
    m.info = dict(workload="srr_array", nx=nx, ny=ny, pitch=pitch)
    return m


def line_bundle_c3(seed=0, n_lines=200, a_tri=1.5e-12, n_y=20, n_z=10,
                   pitch_y=10 * UM, pitch_z=8 * UM):
    """200 parallel lines along x on a 20 x 10 lattice; lengths log-uniform 10-500 um."""
    rng = np.random.default_rng(seed)
    parts, lines = [], []
    for k in range(n_lines):
        l = math.exp(rng.uniform(math.log(10.0), math.log(500.0))) * UM
        w, h = rng.uniform(1.0, 4.0, size=2) * UM
        area = 2.0 * (l * w + l * h + w * h)
        t = int(np.clip(round(area / a_tri), 100, 5000))
        div = box_divisions((l, w, h), t)
        iy, iz = k % n_y, k // n_y
        origin = (0.0, iy * pitch_y, iz * pitch_z)
        parts.append(box_mesh(origin, (l, w, h), div))
        lines.append(dict(origin=origin, size=(l, w, h), div=div))
    m = merge(parts)
    m.info = dict(workload="line_bundle", seed=seed, lines=lines)
    return m


def line_end_ports(mesh, lines):
    """Lumped ports at both ends of the given lines of a line bundle: the vertex ring one
    division in from each end, axis along the line (+x), as (obj, point, axis, radius)."""
    out = []
    for k in lines:
        ln = mesh.info["lines"][k]
        (x0, y0, z0), (l, w, h), (nx, _, _) = ln["origin"], ln["size"], ln["div"]
        if nx < 2:
            raise ValueError("line %d has no vertex ring inside it" % k)
        for x in (x0 + l / nx, x0 + l * (nx - 1) / nx):
            out.append((k, (x, y0 + w / 2, z0 + h / 2), (1.0, 0.0, 0.0), max(w, h)))
    return out


def conductors_c5(seed=0, n_obj=2000, scale=76.0, alpha=1.2, t_min=50, t_max=20000,
                  a_tri=1.5e-12, cube=512 * UM, gap=4 * UM):
    """2000 conductors, triangle counts Pareto(alpha=1.2, scale 76) clipped to 50-20000.

    Bars of cross-section U[1,4] um for t <= 5000; thin square plates (aspect <= 50)
    above.  Shelf-packed into a 512 um cube with gaps of at least 4 um.
    """
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 1.0, size=n_obj)
    t = np.clip(np.round(scale * u ** (-1.0 / alpha)), t_min, t_max).astype(np.int64)
    sizes, divs = [], []
    for ti in t:
        w, h = rng.uniform(1.0, 4.0, size=2) * UM
        area = float(ti) * a_tri
        l = (area / 2.0 - w * h) / (w + h)
        if l <= 250 * UM:
            sz = (max(l, w), w, h)
        else:
            # thin square plate: 2 s^2 + 4 s h = area, aspect s / h <= 50
            for _ in range(3):
                s_ = (-4.0 * h + math.sqrt(16.0 * h * h + 8.0 * area)) / 4.0
                h = max(h, s_ / 50.0)
            sz = (s_, s_, h)
        sizes.append(sz)
        divs.append(box_divisions(sz, int(ti)))
    # shelf packing: sort by height then footprint, fill rows along x, rows along y, layers along z
    order = sorted(range(n_obj), key=lambda i: (-sizes[i][2], -sizes[i][1], -sizes[i][0]))
    pos = [None] * n_obj
    x = y = z = 0.0
    row_h = row_w = 0.0
    layer_h = 0.0
    for i in order:
        l, w, h = sizes[i]
        if x + l > cube:
            x = 0.0
            y += row_w + gap
            row_w = 0.0
        if y + w > cube:
            y = 0.0
            x = 0.0
            z += layer_h + gap
            layer_h = 0.0
            row_w = 0.0
        if z + h > cube:
            raise ValueError("conductors do not fit the packing cube")
        pos[i] = (x, y, z)
        x += l + gap
        row_w = max(row_w, w)
        layer_h = max(layer_h, h)
    # spread the layers evenly over the cube height
    layers = sorted({p[2] for p in pos})
    top = max(pos[i][2] + sizes[i][2] for i in range(n_obj))
    spare = (cube - top) / max(len(layers) - 1, 1)
    lift = {zl: k * spare for k, zl in enumerate(layers)}
    pos = [(p[0], p[1], p[2] + lift[p[2]]) for p in pos]
    parts = [box_mesh(pos[i], sizes[i], divs[i]) for i in range(n_obj)]
    m = merge(parts)
    m.info = dict(workload="conductors", seed=seed, n_obj=n_obj)
    return m


def random_complex(n, seed=0):
    """Complex vector with independent N(0,1) real and imaginary parts."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


WORKLOADS = {
    "bar": bar_c1,
    "small_boxes": small_boxes,
    "srr_array": srr_array_c2,
    "line_bundle": line_bundle_c3,
    "conductors": conductors_c5,
}
