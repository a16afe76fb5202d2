"""Stabilized mean-pressure projection (Ch.3, Sec. Solution of the Eulerian
equations: eq:pressure-projection-smooth and eq:velocity-correction) with
linear finite elements on the triangles.

TEST INFRASTRUCTURE ONLY: like the rest of oracle/, this module is loaded by
the tests, the smoke check and the CPU timing leg of the benchmark, never by
the product path.  FP64; the linear system is solved exactly by SciPy's
sparse direct solver (standing in for the paper's Jacobi-preconditioned
conjugate gradients, whose converged result it is).

Readings.  The mean pressure is P = x . G + P', G the imposed mean gradient
(the input field grad<P>/rho) and P' the solved part, periodic across
identified nodes.  With rho = 1, per step:

    K dP = -(d + C_p K P'^n) / dt,   d_a = sum_e (A_e / 3) div_e(<U>*),

the weak form of eq:pressure-projection-smooth with K the stiffness matrix
over the master nodes and div_e the element divergence of the nodal <U>*.

Walls carry the Neumann condition of eq:wall-pressure-condition, the normal
component of the mean-momentum equation eq:Reynolds at a wall:
    dP/dn = g = nu lap<U_i> n_i - d<u_i u_j>/dx_j n_i
(n the outward unit normal; on wall-function walls also - <U_j> d<U_i>/dx_j n_i),
evaluated from the statistics the projection corrects (the estimate after
the velocity prediction): the nodal Laplacians at the edge's ends and the
element gradients of the nodal Reynolds stresses of the edge's element.  With
B(q)_a = the integral over the wall edges of N_a q (q linear along an edge:
L (2 q_a + q_b) / 6 at end a), the weak form of the step is
    K dP = -(d + C_p K P'^n)/dt + (C_p/dt) B(g^n - G.n) + B(g^{n+1} - g^n),
where g^n is the data that P^n satisfies (the previous step's g; G.n before
the first step, when P' = 0): the new pressure takes the new data, dP the
change of the data, and the stabilizing Laplacian of P'^n the flux of P'^n.
Without walls the boundary terms vanish.  The right-hand side is made
compatible by subtracting its mean over the master nodes, and dP has zero
mean there.  Each particle's velocity then changes by -dt grad(dP) of its
element (eq:velocity-correction applied to the particles), P' += dP, and the
gradient used by the next step's velocity prediction is G plus the average
over the surrounding elements of the element gradients of P'.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def shape_gradients(mesh):
    p = mesh.node_xy[mesh.elem_nodes]
    xBA, yBA = p[:, 1, 0] - p[:, 0, 0], p[:, 1, 1] - p[:, 0, 1]
    xCA, yCA = p[:, 2, 0] - p[:, 0, 0], p[:, 2, 1] - p[:, 0, 1]
    twoA = xBA * yCA - xCA * yBA
    dNdx = np.stack([(yBA - yCA), yCA, -yBA], 1) / twoA[:, None]
    dNdy = np.stack([(xCA - xBA), -xCA, xBA], 1) / twoA[:, None]
    return 0.5 * twoA, dNdx, dNdy


def stiffness(mesh):
    A, dNdx, dNdy = shape_gradients(mesh)
    K = A[:, None, None] * (dNdx[:, :, None] * dNdx[:, None, :] + dNdy[:, :, None] * dNdy[:, None, :])
    mk = mesh.node_master[mesh.elem_nodes]
    rows = np.repeat(mk, 3, axis=1).ravel()
    cols = np.tile(mk, (1, 3)).ravel()
    nn = mesh.n_nodes
    return sp.csr_matrix((K.ravel(), (rows, cols)), shape=(nn, nn))


def elem_gradient(mesh, f):
    """Element gradient of a nodal field (values at the masters), (ne, 2)."""
    _, dNdx, dNdy = shape_gradients(mesh)
    fv = f[mesh.node_master[mesh.elem_nodes]]
    return np.stack([(dNdx * fv).sum(1), (dNdy * fv).sum(1)], 1)


def node_gradient(mesh, f):
    """Average over the elements around each master of their gradients, (2, nn)."""
    g = elem_gradient(mesh, f)
    nn = mesh.n_nodes
    acc = np.zeros((2, nn))
    cnt = np.zeros(nn)
    for e, nodes in enumerate(mesh.node_master[mesh.elem_nodes]):
        for q in np.unique(nodes):
            acc[:, q] += g[e]
            cnt[q] += 1
    out = np.divide(acc, cnt, out=np.zeros_like(acc), where=cnt > 0)
    return out[:, mesh.node_master]


BC_PERIODIC, BC_WALLFN, BC_OUTFLOW = 1, 4, 5


def wall_edges(mesh):
    """Every wall edge (not periodic, not outflow): its end nodes a, b (local nodes k+1
    and k+2 of its element, so the domain lies on its left), its element, its
    outward unit normal and its length, as arrays."""
    keep = np.flatnonzero((mesh.bedge_type != BC_PERIODIC) & (mesh.bedge_type != BC_OUTFLOW))
    e = mesh.bedge_elem[keep]
    k = mesh.bedge_local[keep]
    a = mesh.elem_nodes[e, (k + 1) % 3]
    b = mesh.elem_nodes[e, (k + 2) % 3]
    d = mesh.node_xy[b] - mesh.node_xy[a]
    L = np.sqrt(d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1])
    n = np.stack([d[:, 1], -d[:, 0]], 1) / L[:, None]
    return dict(a=a, b=b, e=e, n=n, L=L, wallfn=mesh.bedge_type[keep] == BC_WALLFN)


def neumann_data(mesh, stats, nu, edges=None):
    """g = nu lap<U_i> n_i - d<u_i u_j>/dx_j n_i (minus <U_j> d<U_i>/dx_j n_i
    on wall-function edges) at both ends of every wall edge, (2, n_edges)."""
    W = wall_edges(mesh) if edges is None else edges
    mk = mesh.node_master
    _, dNdx, dNdy = shape_gradients(mesh)
    em = mk[mesh.elem_nodes[W["e"]]]

    def grad(field):  # element gradient of a nodal field on the edges' elements
        v = stats[field][em]
        return (dNdx[W["e"]] * v).sum(1), (dNdy[W["e"]] * v).sum(1)

    R11x, R11y = grad(5)
    R22x, R22y = grad(6)
    R12x, R12y = grad(8)
    divR = np.stack([R11x + R12y, R12x + R22y], 1)
    nx, ny = W["n"][:, 0], W["n"][:, 1]
    out = []
    for end in ("a", "b"):
        q = mk[W[end]]
        g = nu * (stats[21][q] * nx + stats[22][q] * ny) - (divR[:, 0] * nx + divR[:, 1] * ny)
        if W["wallfn"].any():
            Ux, Uy = grad(0)
            Vx, Vy = grad(1)
            U, V = stats[0][q], stats[1][q]
            adv = np.stack([U * Ux + V * Uy, U * Vx + V * Vy], 1)
            g = g - np.where(W["wallfn"], adv[:, 0] * nx + adv[:, 1] * ny, 0.0)
        out.append(g)
    return np.array(out)


def boundary_vector(mesh, g, edges=None):
    """B(q)_a: the integral over the wall edges of N_a q, q linear along each
    edge with values g[0] at its start and g[1] at its end; over the masters."""
    W = wall_edges(mesh) if edges is None else edges
    mk = mesh.node_master
    B = np.zeros(mesh.n_nodes)
    np.add.at(B, mk[W["a"]], W["L"] * (2.0 * g[0] + g[1]) / 6.0)
    np.add.at(B, mk[W["b"]], W["L"] * (g[0] + 2.0 * g[1]) / 6.0)
    return B


def imposed_normal(mesh, G, edges=None):
    """G.n at both ends of every wall edge, G the nodal imposed gradient (2, nn)."""
    W = wall_edges(mesh) if edges is None else edges
    mk = mesh.node_master
    return np.array([G[0][mk[W[end]]] * W["n"][:, 0] + G[1][mk[W[end]]] * W["n"][:, 1] for end in ("a", "b")])


def solve_dp(mesh, U, V, P, dt, Cp, flux=None):
    """dP at every node from the nodal <U>*, <V>* and P'^n; flux (nn) is the
    wall boundary term added to the right-hand side (None: natural
    conditions)."""
    A, dNdx, dNdy = shape_gradients(mesh)
    mk = mesh.node_master[mesh.elem_nodes]
    div = (dNdx * U[mk]).sum(1) + (dNdy * V[mk]).sum(1)
    nn = mesh.n_nodes
    d = np.zeros(nn)
    np.add.at(d, mk.ravel(), np.repeat(A / 3.0 * div, 3))
    K = stiffness(mesh)
    masters = np.unique(mesh.node_master)
    b = -(d + Cp * (K @ P[mesh.node_master])) / dt
    if flux is not None:
        b = b + flux
    b[masters] -= b[masters].mean()
    # the solution is unique up to a constant: pin the first master, then
    # take the zero-mean representative
    free = masters[1:]
    x = np.zeros(nn)
    x[free] = spla.spsolve(K[free][:, free].tocsc(), b[free])
    x[masters] -= x[masters].mean()
    return x[mesh.node_master]
