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
over the master nodes, div_e the element divergence of the nodal <U>*, and
natural (zero normal flux) conditions for both dP and the stabilizing
Laplacian of P'^n at walls.  The right-hand side is made compatible by
subtracting its mean over the master nodes, and dP has zero mean there.  Each
particle's velocity then changes by -dt grad(dP) of its element
(eq:velocity-correction applied to the particles), P' += dP, and the
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


def solve_dp(mesh, U, V, P, dt, Cp):
    """dP at every node from the nodal <U>*, <V>* and P'^n."""
    A, dNdx, dNdy = shape_gradients(mesh)
    mk = mesh.node_master[mesh.elem_nodes]
    div = (dNdx * U[mk]).sum(1) + (dNdy * V[mk]).sum(1)
    nn = mesh.n_nodes
    d = np.zeros(nn)
    np.add.at(d, mk.ravel(), np.repeat(A / 3.0 * div, 3))
    K = stiffness(mesh)
    masters = np.unique(mesh.node_master)
    b = -(d + Cp * (K @ P[mesh.node_master])) / dt
    b[masters] -= b[masters].mean()
    # the solution is unique up to a constant: pin the first master, then
    # take the zero-mean representative
    free = masters[1:]
    x = np.zeros(nn)
    x[free] = spla.spsolve(K[free][:, free].tocsc(), b[free])
    x[masters] -= x[masters].mean()
    return x[mesh.node_master]
