"""Elliptic relaxation for the tensor wp_ij (eq:elliptic-relaxation-Lagrangian
with eq:L and eq:Cxi, and the wall condition wp_ij = -4.5 eps n_i n_j of the
near-wall section of Ch.2), solved with linear finite elements on the
triangles (Ch.3, Sec. Solution of the Eulerian equations).

TEST INFRASTRUCTURE ONLY: like the rest of oracle/, this module is loaded by
the tests, the smoke check and the CPU timing leg of the benchmark, never by
the product path.  FP64; the linear systems are solved exactly by SciPy's
sparse direct solver (a library primitive standing in for the paper's
Jacobi-preconditioned conjugate gradients, whose converged result it is).

Per component ij, over the master nodes (periodic identification):

    sum_e [ M_e + L2_{e,ij} K_e ] wp_ij = sum_e M_e f_ij

M_e is the consistent mass matrix (A/12)(1 + delta_ab), K_e the stiffness
matrix A grad N_a . grad N_b, f_ij the nodal right-hand side of
eq:elliptic-relaxation-Lagrangian (its local form).  L2_{e,ij} = L_ij^2 with
eq:L evaluated from the element averages of the nodal statistics:
k = max(<u_i u_i>/2, k_floor), eps = <omega>(k + nu C_T^2 <omega>), and
C_xi,ij = 1 + 1.3 n_i n_j (eq:Cxi, read so that only wp_22 changes next to a
wall along x), n the outward unit normal of the no-slip wall edge closest to
the element's centroid (n = 0 without such walls, the lowest edge number on
ties); L2 = 0 where eps <= 0.  Dirichlet condition at the nodes of no-slip
edges: wp_ij = -4.5 eps n_i n_j with the node's eps and n the normalised sum
of the outward unit normals of its no-slip edges; elsewhere the natural
condition (no normal flux).  Parity: pinned by tests/test_oracle_elliptic.py.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

BC_NOSLIP = 3


def _edge_nodes(mesh, b):
    e, k = mesh.bedge_elem[b], mesh.bedge_local[b]
    return mesh.elem_nodes[e, (k + 1) % 3], mesh.elem_nodes[e, (k + 2) % 3]


def wall_geometry(mesh):
    """No-slip wall edges: endpoints (nw, 2, 2) and outward unit normals (nw, 2)."""
    walls = np.nonzero(mesh.bedge_type == BC_NOSLIP)[0]
    P = np.zeros((walls.size, 2, 2))
    N = np.zeros((walls.size, 2))
    for j, b in enumerate(walls):
        a, c = _edge_nodes(mesh, b)
        A, B = mesh.node_xy[a], mesh.node_xy[c]
        d = B - A
        P[j] = A, B
        N[j] = np.array([d[1], -d[0]]) / np.hypot(d[0], d[1])  # the domain lies on the edge's left
    return walls, P, N


def element_normals(mesh):
    """Outward normal of the no-slip wall edge closest to each element's centroid."""
    walls, P, N = wall_geometry(mesh)
    ne = mesh.n_elems
    if walls.size == 0:
        return np.zeros((ne, 2))
    cen = mesh.node_xy[mesh.elem_nodes].sum(1) / 3.0
    A, B = P[:, 0], P[:, 1]
    d = B - A
    t = ((cen[:, None, :] - A[None]) * d[None]).sum(-1) / (d * d).sum(-1)[None]
    t = np.clip(t, 0.0, 1.0)
    q = A[None] + t[..., None] * d[None]
    dist2 = ((cen[:, None, :] - q) ** 2).sum(-1)
    return N[np.argmin(dist2, axis=1)]  # argmin takes the first (lowest edge) on ties


def wall_nodes(mesh):
    """Master nodes on no-slip edges and their unit normals (sum of the unit
    outward normals of the node's no-slip edges, normalised)."""
    walls, P, N = wall_geometry(mesh)
    acc = {}
    for j, b in enumerate(walls):
        for n in _edge_nodes(mesh, b):
            q = int(mesh.node_master[n])
            acc[q] = acc.get(q, np.zeros(2)) + N[j]
    nodes = np.array(sorted(acc), dtype=np.int64)
    nv = np.array([acc[q] / np.hypot(*acc[q]) for q in nodes]).reshape(-1, 2)
    return nodes, nv


def _k_eps(params, R, Om):
    k = 0.5 * (R[0] + R[1] + R[2])
    k = np.where(k > params["k_floor"], k, params["k_floor"])
    eps = Om * (k + params["nu"] * params["CT"] ** 2 * Om)
    return k, eps


def element_L2(mesh, params, stats):
    """L_ij^2 per element, (ne, 3, 3)."""
    mk = mesh.node_master[mesh.elem_nodes]
    R = stats[5:8][:, mk].sum(-1) / 3.0
    Om = stats[3][mk].sum(-1) / 3.0
    k, eps = _k_eps(params, R, Om)
    n2 = np.zeros((mesh.n_elems, 3))
    n2[:, :2] = element_normals(mesh)
    ok = eps > 0.0
    epsok = np.where(ok, eps, 1.0)
    L2 = np.zeros((mesh.n_elems, 3, 3))
    for i in range(3):
        for j in range(3):
            cxi = 1.0 + 1.3 * n2[:, i] * n2[:, j]
            L = params["CL"] * np.maximum(cxi * k ** 1.5 / epsok,
                                          params["Ceta"] * (params["nu"] ** 3 / epsok) ** 0.25)
            L2[:, i, j] = np.where(ok, L * L, 0.0)
    return L2


def _local_matrices(mesh):
    p = mesh.node_xy[mesh.elem_nodes]
    xBA, yBA = p[:, 1, 0] - p[:, 0, 0], p[:, 1, 1] - p[:, 0, 1]
    xCA, yCA = p[:, 2, 0] - p[:, 0, 0], p[:, 2, 1] - p[:, 0, 1]
    twoA = xBA * yCA - xCA * yBA
    A = 0.5 * twoA
    dNdx = np.stack([(yBA - yCA), yCA, -yBA], 1) / twoA[:, None]
    dNdy = np.stack([(xCA - xBA), -xCA, xBA], 1) / twoA[:, None]
    K = A[:, None, None] * (dNdx[:, :, None] * dNdx[:, None, :] + dNdy[:, :, None] * dNdy[:, None, :])
    Mm = A[:, None, None] / 12.0 * (np.ones((3, 3)) + np.eye(3))[None]
    return Mm, K


def solve(mesh, params, stats, f, L2=None):
    """wp (9, nn) from the nodal right-hand side f (9, nn) and the statistics."""
    nn = mesh.n_nodes
    mk = mesh.node_master[mesh.elem_nodes]
    Mm, K = _local_matrices(mesh)
    if L2 is None:
        L2 = element_L2(mesh, params, stats)
    rows = np.repeat(mk, 3, axis=1).ravel()
    cols = np.tile(mk, (1, 3)).ravel()
    Mg = sp.csr_matrix((Mm.ravel(), (rows, cols)), shape=(nn, nn))
    dn, dnv = wall_nodes(mesh)
    k_n, eps_n = _k_eps(params, stats[5:8], stats[3])
    masters = np.unique(mesh.node_master)
    free = np.setdiff1d(masters, dn)
    wp = np.zeros((9, nn))
    for i in range(3):
        for j in range(3):
            c = 3 * i + j
            Ag = sp.csr_matrix(((Mm + L2[:, i, j][:, None, None] * K).ravel(), (rows, cols)), shape=(nn, nn))
            fm = f[c][mesh.node_master]  # masters' values
            b = Mg @ fm
            x = np.zeros(nn)
            if dn.size:
                ni = dnv[:, i] if i < 2 else np.zeros(dn.size)
                nj = dnv[:, j] if j < 2 else np.zeros(dn.size)
                x[dn] = -4.5 * eps_n[dn] * ni * nj
            rhs = b[free] - Ag[free][:, dn] @ x[dn] if dn.size else b[free]
            x[free] = spla.spsolve(Ag[free][:, free].tocsc(), rhs)
            wp[c] = x[mesh.node_master]
    return wp
