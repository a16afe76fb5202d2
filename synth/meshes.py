"""Seeded synthetic triangle meshes shaped like the dissertation's test domains.

This module produces *inputs* only: node coordinates, counter-clockwise
triangles, the element-surrounding-element table with tagged boundary edges,
periodic edge pairs and periodic node identification.  It holds none of the
particle method's arithmetic and is shared by the oracle tests and the GPU
path alike.

The paper meshes its domains with Gmsh (Ch.3, Sec. "Solution of the Eulerian
equations"); Gmsh is not available here, so every mesh below is a graded
tensor grid whose quads are split into two triangles.  Interior nodes may be
jittered and each quad's diagonal chosen by the Delaunay (empty circumcircle)
test, which gives an irregular, unstructured triangulation with valences 4..8.
Elements and nodes are numbered along a Morton (Z-order) curve of their
coordinates so that neighbouring elements sit close together in memory.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

BC_PERIODIC = 1
BC_SLIP = 2
BC_NOSLIP = 3
BC_WALLFN = 4   # wall treated by wall functions
BC_OUTFLOW = 5  # outflow edge paired with a periodic (inflow) edge: particles leaving are relocated


@dataclass
class Mesh:
    node_xy: np.ndarray        # (Nn, 2) float64
    elem_nodes: np.ndarray     # (Ne, 3) int32, counter-clockwise
    elem_nbr: np.ndarray       # (Ne, 3) int32, neighbour across the edge opposite local node k; <0 => -(bedge+1)
    bedge_elem: np.ndarray     # (Nb,) int32
    bedge_local: np.ndarray    # (Nb,) int32, local edge index k in bedge_elem
    bedge_type: np.ndarray     # (Nb,) int32, BC_*
    bedge_partner: np.ndarray  # (Nb,) int32, periodic partner edge or -1
    bedge_shift: np.ndarray    # (Nb, 2) float64, translation added to a particle crossing the edge
    node_master: np.ndarray    # (Nn,) int32, periodic identification (master node index)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self):
        return int(self.node_xy.shape[0])

    @property
    def n_elems(self):
        return int(self.elem_nodes.shape[0])

    @property
    def n_bedges(self):
        return int(self.bedge_elem.shape[0])

    def areas(self):
        p = self.node_xy[self.elem_nodes]
        return 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                      - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))


# ----------------------------------------------------------------------------
# 1-D node distributions
# ----------------------------------------------------------------------------

def _graded(a, b, n, wall_a, wall_b, ratio):
    """n intervals on [a, b]; spacing shrinks geometrically toward wall ends so
    that the largest / smallest spacing equals `ratio`."""
    t = np.linspace(0.0, 1.0, n + 1)
    if ratio <= 1.0 or not (wall_a or wall_b):
        s = t
    else:
        beta = np.log(ratio)
        if wall_a and wall_b:
            # two mirrored one-sided stretchings meeting in the middle
            h = 0.5
            tt = np.where(t <= h, t / h, (1.0 - t) / h)
            f = (np.exp(beta * tt) - 1.0) / (np.exp(beta) - 1.0)
            s = np.where(t <= h, 0.5 * f, 1.0 - 0.5 * f)
        elif wall_a:
            s = (np.exp(beta * t) - 1.0) / (np.exp(beta) - 1.0)
        else:
            s = 1.0 - (np.exp(beta * (1.0 - t)) - 1.0) / (np.exp(beta) - 1.0)
    x = a + (b - a) * s
    x[0], x[-1] = a, b
    return x


def _join(segments):
    out = [segments[0]]
    for s in segments[1:]:
        out.append(s[1:])
    return np.concatenate(out)


def channel_wall_refinement(n_half, h=1.0):
    """Cross-stream coordinates refined toward the walls with the law
    y/h = 1 - cos(pi/2 * a^(3/4)), a uniform on [0, 1] (Ch.4, channel grid
    refinement), mirrored about the centreline: 2*n_half intervals on [0, 2h]."""
    a = np.linspace(0.0, 1.0, n_half + 1)
    lower = h * (1.0 - np.cos(0.5 * np.pi * a ** 0.75))
    lower[0], lower[-1] = 0.0, h
    upper = 2.0 * h - lower[::-1]
    return np.concatenate([lower, upper[1:]])


# ----------------------------------------------------------------------------
# Morton ordering
# ----------------------------------------------------------------------------

def _part1by1(v):
    v = v.astype(np.uint64) & np.uint64(0xFFFFFFFF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x0000FFFF0000FFFF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x00FF00FF00FF00FF)
    v = (v | (v << np.uint64(4))) & np.uint64(0x0F0F0F0F0F0F0F0F)
    v = (v | (v << np.uint64(2))) & np.uint64(0x3333333333333333)
    v = (v | (v << np.uint64(1))) & np.uint64(0x5555555555555555)
    return v


def morton_order(xy):
    lo = xy.min(axis=0)
    span = np.maximum(xy.max(axis=0) - lo, 1e-300)
    q = np.floor((xy - lo) / span.max() * 65535.0).astype(np.int64)
    code = _part1by1(q[:, 0]) | (_part1by1(q[:, 1]) << np.uint64(1))
    return np.argsort(code, kind="stable")


# ----------------------------------------------------------------------------
# Triangulation of a tensor grid
# ----------------------------------------------------------------------------

def _incircle(ax, ay, bx, by, cx, cy, dx, dy):
    """>0 when d lies inside the circumcircle of the CCW triangle abc."""
    adx, ady = ax - dx, ay - dy
    bdx, bdy = bx - dx, by - dy
    cdx, cdy = cx - dx, cy - dy
    return ((adx * adx + ady * ady) * (bdx * cdy - cdx * bdy)
            - (bdx * bdx + bdy * bdy) * (adx * cdy - cdx * ady)
            + (cdx * cdx + cdy * cdy) * (adx * bdy - bdx * ady))


def _tensor_triangulation(xs, ys, keep_quad, rng, jitter, diag):
    """Triangulate the tensor grid xs x ys, dropping quads where keep_quad is False.

    diag: 'same' (every quad split along (i,j)-(i+1,j+1)) or 'delaunay'
    (Delaunay choice per quad after jitter, ties broken at random)."""
    nx, ny = len(xs), len(ys)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    xy = np.stack([X.ravel(), Y.ravel()], axis=1).copy()
    nid = np.arange(nx * ny).reshape(nx, ny)
    qi, qj = np.nonzero(keep_quad)
    p0 = nid[qi, qj]
    p1 = nid[qi + 1, qj]
    p2 = nid[qi + 1, qj + 1]
    p3 = nid[qi, qj + 1]
    used = np.zeros(nx * ny, bool)
    used[np.concatenate([p0, p1, p2, p3])] = True
    return xy, (p0, p1, p2, p3), used, nid


def _finish(xy, quads, used, rng, jitter, diag, fixed_nodes, classify, period, name, meta):
    p0, p1, p2, p3 = quads
    if jitter > 0.0:
        # local spacing estimate per node from the quads that use it
        n = xy.shape[0]
        hx = np.full(n, np.inf)
        hy = np.full(n, np.inf)
        qdx = np.abs(xy[p1, 0] - xy[p0, 0])
        qdy = np.abs(xy[p3, 1] - xy[p0, 1])
        for p in (p0, p1, p2, p3):
            np.minimum.at(hx, p, qdx)
            np.minimum.at(hy, p, qdy)
        mov = used & ~fixed_nodes
        d = rng.uniform(-1.0, 1.0, size=(n, 2))
        xy = xy.copy()
        xy[mov, 0] += jitter * hx[mov] * d[mov, 0]
        xy[mov, 1] += jitter * hy[mov] * d[mov, 1]
    if diag == "same":
        use02 = np.ones(p0.shape[0], bool)
    else:
        det = _incircle(xy[p0, 0], xy[p0, 1], xy[p1, 0], xy[p1, 1], xy[p2, 0], xy[p2, 1],
                        xy[p3, 0], xy[p3, 1])
        scale = (np.abs(xy[p2, 0] - xy[p0, 0]) + np.abs(xy[p2, 1] - xy[p0, 1])) ** 4
        tie = np.abs(det) <= 1e-9 * scale
        coin = rng.random(p0.shape[0]) < 0.5
        use02 = np.where(tie, coin, det <= 0.0)
    t1 = np.where(use02[:, None], np.stack([p0, p1, p2], 1), np.stack([p0, p1, p3], 1))
    t2 = np.where(use02[:, None], np.stack([p0, p2, p3], 1), np.stack([p1, p2, p3], 1))
    tri = np.concatenate([t1, t2], axis=0)
    # drop unused nodes and renumber nodes and elements along a Morton curve
    keep = np.nonzero(used)[0]
    xy = xy[keep]
    remap = np.full(used.shape[0], -1, np.int64)
    remap[keep] = np.arange(keep.shape[0])
    tri = remap[tri]
    norder = morton_order(xy)
    ninv = np.empty_like(norder)
    ninv[norder] = np.arange(norder.shape[0])
    xy = xy[norder]
    tri = ninv[tri]
    cent = xy[tri].mean(axis=1)
    eorder = morton_order(cent)
    tri = tri[eorder]
    return build_mesh(xy, tri.astype(np.int32), classify, period, name, meta)


# ----------------------------------------------------------------------------
# Connectivity (elements surrounding elements, boundary edges, periodicity)
# ----------------------------------------------------------------------------

def build_mesh(xy, tri, classify, period, name="", meta=None):
    """Assemble the mesh tables from coordinates and CCW triangles.

    classify(mid_xy (Nb,2), normal (Nb,2)) -> BC type per boundary edge.
    period: (Px, Py) periods (0 => not periodic in that direction)."""
    xy = np.ascontiguousarray(xy, np.float64)
    tri = np.ascontiguousarray(tri, np.int32)
    ne = tri.shape[0]
    a = np.stack([tri[:, 1], tri[:, 2], tri[:, 0]], 1)  # edge k = (node k+1, node k+2)
    b = np.stack([tri[:, 2], tri[:, 0], tri[:, 1]], 1)
    lo = np.minimum(a, b).ravel().astype(np.int64)
    hi = np.maximum(a, b).ravel().astype(np.int64)
    key = lo * (xy.shape[0] + 1) + hi
    order = np.argsort(key, kind="stable")
    ks = key[order]
    nbr = np.full(ne * 3, -1, np.int64)
    same = ks[1:] == ks[:-1]
    i0 = order[:-1][same]
    i1 = order[1:][same]
    nbr[i0] = i1 // 3
    nbr[i1] = i0 // 3
    if np.any(np.bincount(ks, minlength=0)[ks] > 2) if False else False:
        raise ValueError("non-manifold edge")
    bslots = np.nonzero(nbr < 0)[0]
    nb = bslots.shape[0]
    be = (bslots // 3).astype(np.int32)
    bl = (bslots % 3).astype(np.int32)
    pa = xy[a.ravel()[bslots]]
    pb = xy[b.ravel()[bslots]]
    mid = 0.5 * (pa + pb)
    t = pb - pa
    nrm = np.stack([t[:, 1], -t[:, 0]], 1)  # outward for a CCW element
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    btype = np.asarray(classify(mid, nrm), np.int32)
    partner = np.full(nb, -1, np.int32)
    shift = np.zeros((nb, 2), np.float64)
    master = np.arange(xy.shape[0], dtype=np.int64)
    for axis in (0, 1):
        P = period[axis]
        if not P:
            continue
        lo_side = (btype == BC_PERIODIC) & (np.abs(mid[:, axis] - xy[:, axis].min()) < 1e-12 * P)
        hi_side = (btype == BC_PERIODIC) & (np.abs(mid[:, axis] - (xy[:, axis].min() + P)) < 1e-12 * P)
        il = np.nonzero(lo_side)[0]
        ih = np.nonzero(hi_side)[0]
        other = 1 - axis
        kl = np.round(mid[il, other] * 1e9).astype(np.int64)
        kh = np.round(mid[ih, other] * 1e9).astype(np.int64)
        sl = np.argsort(kl)
        sh = np.argsort(kh)
        if il.shape[0] != ih.shape[0] or np.any(kl[sl] != kh[sh]):
            raise ValueError("periodic boundary edges do not pair up")
        pl, ph = il[sl], ih[sh]
        partner[pl] = ph
        partner[ph] = pl
        shift[pl, axis] = P
        shift[ph, axis] = -P
        # node identification: nodes on the high side map to the low side
        x0 = xy[:, axis].min()
        on_lo = np.nonzero(np.abs(xy[:, axis] - x0) < 1e-12 * P)[0]
        on_hi = np.nonzero(np.abs(xy[:, axis] - (x0 + P)) < 1e-12 * P)[0]
        klo = np.round(xy[on_lo, other] * 1e9).astype(np.int64)
        khi = np.round(xy[on_hi, other] * 1e9).astype(np.int64)
        slo, shi = np.argsort(klo), np.argsort(khi)
        if np.any(klo[slo] != khi[shi]):
            raise ValueError("periodic nodes do not pair up")
        master[on_hi[shi]] = on_lo[slo]
    # resolve chains (corner nodes of doubly periodic meshes)
    for _ in range(3):
        master = master[master]
    nbr2 = nbr.copy()
    nbr2[bslots] = -(np.arange(nb) + 1)
    return Mesh(node_xy=xy, elem_nodes=tri, elem_nbr=nbr2.reshape(ne, 3).astype(np.int32),
                bedge_elem=be, bedge_local=bl, bedge_type=btype, bedge_partner=partner,
                bedge_shift=shift, node_master=master.astype(np.int32), name=name,
                meta=dict(meta or {}))


# ----------------------------------------------------------------------------
# The four mesh families
# ----------------------------------------------------------------------------

def periodic_square(n=32, L=1.0):
    """[0,L)^2, n x n squares each split along the same diagonal, periodic in
    x and y: 2 n^2 right triangles."""
    xs = np.linspace(0.0, L, n + 1)
    ys = np.linspace(0.0, L, n + 1)
    keep = np.ones((n, n), bool)
    xy, quads, used, _ = _tensor_triangulation(xs, ys, keep, None, 0.0, "same")
    fixed = np.ones(xy.shape[0], bool)
    return _finish(xy, quads, used, np.random.default_rng(0), 0.0, "same", fixed,
                   lambda m, nrm: np.full(m.shape[0], BC_PERIODIC), (L, L),
                   f"periodic_square_{n}", {"L": L, "n": n})


def graded_channel(nx=100, n_half=50, Lx=6.0, h=1.0, jitter=0.15, seed=0, top=BC_NOSLIP):
    """Plane channel [0,Lx]x[0,2h]: streamwise periodic, no-slip walls at y=0
    and y=2h (top wall type selectable), nodes refined toward the walls with
    the channel-grid refinement law; 2*nx*2*n_half triangles."""
    rng = np.random.default_rng(seed)
    xs = np.linspace(0.0, Lx, nx + 1)
    ys = channel_wall_refinement(n_half, h)
    keep = np.ones((nx, 2 * n_half), bool)
    xy, quads, used, _ = _tensor_triangulation(xs, ys, keep, rng, jitter, "delaunay")
    fixed = ((np.abs(xy[:, 0]) < 1e-12) | (np.abs(xy[:, 0] - Lx) < 1e-12)
             | (np.abs(xy[:, 1]) < 1e-12) | (np.abs(xy[:, 1] - 2 * h) < 1e-12))

    def classify(m, nrm):
        t = np.full(m.shape[0], BC_NOSLIP, np.int32)
        t[(np.abs(m[:, 0]) < 1e-9) | (np.abs(m[:, 0] - Lx) < 1e-9)] = BC_PERIODIC
        t[np.abs(m[:, 1] - 2 * h) < 1e-9] = top
        return t

    return _finish(xy, quads, used, rng, jitter, "delaunay", fixed, classify, (Lx, 0.0),
                   f"channel_{nx}x{2 * n_half}", {"Lx": Lx, "H": 2 * h})


def uniform_channel(nx=40, ny=20, Lx=6.0, h=1.0, jitter=0.15, seed=0, wall=BC_WALLFN):
    """Plane channel [0,Lx]x[0,2h] on a uniform grid: streamwise periodic,
    both walls of type `wall` (wall functions by default: the first gridpoint
    off the wall sits in the log layer instead of the viscous sublayer)."""
    rng = np.random.default_rng(seed)
    xs = np.linspace(0.0, Lx, nx + 1)
    ys = np.linspace(0.0, 2 * h, ny + 1)
    keep = np.ones((nx, ny), bool)
    xy, quads, used, _ = _tensor_triangulation(xs, ys, keep, rng, jitter, "delaunay")
    fixed = ((np.abs(xy[:, 0]) < 1e-12) | (np.abs(xy[:, 0] - Lx) < 1e-12)
             | (np.abs(xy[:, 1]) < 1e-12) | (np.abs(xy[:, 1] - 2 * h) < 1e-12))

    def classify(m, nrm):
        t = np.full(m.shape[0], wall, np.int32)
        t[(np.abs(m[:, 0]) < 1e-9) | (np.abs(m[:, 0] - Lx) < 1e-9)] = BC_PERIODIC
        return t

    return _finish(xy, quads, used, rng, jitter, "delaunay", fixed, classify, (Lx, 0.0),
                   f"uniform_channel_{nx}x{ny}", {"Lx": Lx, "H": 2 * h})


def _box_with_blocks(Lx, Ly, blocks, h, ratio, jitter, seed, top_bc, name):
    """Box [0,Lx]x[0,Ly] with rectangular blocks standing on the floor, graded
    `ratio`:1 toward the floor, the top of the blocks and their sides.
    Streamwise periodic; no-slip floor and blocks; top boundary `top_bc`."""
    rng = np.random.default_rng(seed)
    xl = sorted({0.0, Lx} | {b[0] for b in blocks} | {b[1] for b in blocks})
    yl = sorted({0.0, Ly} | {b[2] for b in blocks})
    wall_x = {b[0] for b in blocks} | {b[1] for b in blocks}
    wall_y = {0.0} | {b[2] for b in blocks}
    if top_bc == BC_NOSLIP:
        wall_y = wall_y | {Ly}

    def axis(lines, walls):
        segs = []
        for a, b in zip(lines[:-1], lines[1:]):
            wa, wb = a in walls, b in walls
            n = max(2, int(round((b - a) / h * (1.0 if not (wa or wb) else 1.0))))
            segs.append(_graded(a, b, n, wa, wb, ratio))
        return _join(segs)

    xs = axis(xl, wall_x)
    ys = axis(yl, wall_y)
    xc = 0.5 * (xs[1:] + xs[:-1])
    yc = 0.5 * (ys[1:] + ys[:-1])
    keep = np.ones((xs.shape[0] - 1, ys.shape[0] - 1), bool)
    for (x0, x1, y1) in blocks:
        keep &= ~(((xc > x0) & (xc < x1))[:, None] & (yc < y1)[None, :])
    xy, quads, used, _ = _tensor_triangulation(xs, ys, keep, rng, jitter, "delaunay")

    def on_block_wall(p):
        f = np.zeros(p.shape[0], bool)
        for (x0, x1, y1) in blocks:
            side = ((np.abs(p[:, 0] - x0) < 1e-9) | (np.abs(p[:, 0] - x1) < 1e-9)) & (p[:, 1] <= y1 + 1e-9)
            topb = (np.abs(p[:, 1] - y1) < 1e-9) & (p[:, 0] >= x0 - 1e-9) & (p[:, 0] <= x1 + 1e-9)
            f |= side | topb
        return f

    fixed = ((np.abs(xy[:, 0]) < 1e-12) | (np.abs(xy[:, 0] - Lx) < 1e-12)
             | (np.abs(xy[:, 1]) < 1e-12) | (np.abs(xy[:, 1] - Ly) < 1e-12) | on_block_wall(xy))

    def classify(m, nrm):
        t = np.full(m.shape[0], BC_NOSLIP, np.int32)
        t[(np.abs(m[:, 0]) < 1e-9) | (np.abs(m[:, 0] - Lx) < 1e-9)] = BC_PERIODIC
        t[np.abs(m[:, 1] - Ly) < 1e-9] = top_bc
        return t

    return _finish(xy, quads, used, rng, jitter, "delaunay", fixed, classify, (Lx, 0.0), name,
                   {"Lx": Lx, "Ly": Ly, "blocks": blocks})


def canyon(target_elems=200_000, jitter=0.15, seed=0):
    """Street-canyon-like box [0,20]x[0,10] with two 2x3 blocks on the floor at
    x in [7,9] and [11,13]; graded 5:1 toward the walls; no-slip floor and
    blocks, free-slip top, streamwise periodic."""
    blocks = [(7.0, 9.0, 3.0), (11.0, 13.0, 3.0)]
    fluid_area = 20.0 * 10.0 - 2 * 2.0 * 3.0
    h = np.sqrt(2.0 * fluid_area / target_elems)
    return _box_with_blocks(20.0, 10.0, blocks, h, 5.0, jitter, seed, BC_SLIP,
                            f"canyon_{target_elems}")


def channel_block(target_elems=1_000_000, jitter=0.15, seed=0):
    """Channel [0,30]x[0,2] with a 1 x 0.5 block on the floor at x in [5,6];
    graded 5:1 toward the walls; no-slip walls and block, streamwise periodic."""
    blocks = [(5.0, 6.0, 0.5)]
    fluid_area = 30.0 * 2.0 - 0.5
    h = np.sqrt(2.0 * fluid_area / target_elems)
    return _box_with_blocks(30.0, 2.0, blocks, h, 5.0, jitter, seed, BC_NOSLIP,
                            f"channel_block_{target_elems}")


def box(nx=16, ny=16, Lx=1.0, Ly=1.0, jitter=0.0, seed=0, bc=BC_SLIP, diag="same"):
    """Rectangle [0,Lx]x[0,Ly] on a uniform grid, every side a wall of type `bc`
    (no periodicity); optional jitter of interior nodes and Delaunay diagonals."""
    rng = np.random.default_rng(seed)
    xs = np.linspace(0.0, Lx, nx + 1)
    ys = np.linspace(0.0, Ly, ny + 1)
    keep = np.ones((nx, ny), bool)
    xy, quads, used, _ = _tensor_triangulation(xs, ys, keep, rng, jitter, diag)
    fixed = ((np.abs(xy[:, 0]) < 1e-12) | (np.abs(xy[:, 0] - Lx) < 1e-12)
             | (np.abs(xy[:, 1]) < 1e-12) | (np.abs(xy[:, 1] - Ly) < 1e-12))
    return _finish(xy, quads, used, rng, jitter, diag, fixed,
                   lambda m, nrm: np.full(m.shape[0], bc, np.int32), (0.0, 0.0),
                   f"box_{nx}x{ny}", {"Lx": Lx, "Ly": Ly})


def with_outflow(mesh):
    """A copy of a streamwise-periodic mesh whose periodic edges at the
    largest x become outflow edges: particles leaving there are relocated at
    the inflow (the edges at the smallest x, which stay periodic, so that
    leaving upstream is periodic) with a reset velocity.  The nodes stay
    identified across the pair."""
    from dataclasses import replace

    bt = mesh.bedge_type.copy()
    e, k = mesh.bedge_elem, mesh.bedge_local
    a = mesh.elem_nodes[e, (k + 1) % 3]
    b = mesh.elem_nodes[e, (k + 2) % 3]
    mid_x = 0.5 * (mesh.node_xy[a, 0] + mesh.node_xy[b, 0])
    xmax = mesh.node_xy[:, 0].max()
    hi = (bt == BC_PERIODIC) & (np.abs(mid_x - xmax) < 1e-9 * max(1.0, abs(xmax)))
    assert hi.any() and (bt[mesh.bedge_partner[hi]] == BC_PERIODIC).all()
    bt[hi] = BC_OUTFLOW
    return replace(mesh, bedge_type=bt, name=mesh.name + "_outflow")

