"""FP64 reference of the denoiser network (TEST INFRASTRUCTURE ONLY).

A 4-layer perceptron 48 -> H -> H -> H -> 8, GELU (exact, erf form)
activations, y = x W + b per layer, mean-squared-error loss, written out with
NumPy in float64.  With bf16_storage=True the weights, inputs and the stored
activations and back-propagated errors are rounded to bfloat16 (round to
nearest even) at the same points as the GPU kernels store them, everything
else stays float64.  Also: the nodal features of the plain statistics and the
merge rule with the plain-estimator fallback.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

SQRT1_2 = np.sqrt(0.5)


def bf16(x):
    """Round float64/float32 values to bfloat16 (nearest even), returned as float64."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z * SQRT1_2))


def dgelu(z):
    return 0.5 * (1.0 + erf(z * SQRT1_2)) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def unpack(p, h):
    p = np.asarray(p, np.float64)
    sizes = [(48, h), (h,), (h, h), (h,), (h, h), (h,), (h, 8), (8,)]
    out, o = [], 0
    for s in sizes:
        n = int(np.prod(s))
        out.append(p[o:o + n].reshape(s))
        o += n
    assert o == p.size
    return out


def pack(ts):
    return np.concatenate([np.asarray(t, np.float64).ravel() for t in ts])


def forward(p, h, x, bf16_storage=False):
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(p, h)
    r = bf16 if bf16_storage else (lambda a: np.asarray(a, np.float64))
    X = r(x)
    Z1 = X @ r(W1) + b1
    H1 = r(gelu(Z1))
    Z2 = H1 @ r(W2) + b2
    H2 = r(gelu(Z2))
    Z3 = H2 @ r(W3) + b3
    H3 = r(gelu(Z3))
    Y = H3 @ r(W4) + b4
    return Y, (X, Z1, H1, Z2, H2, Z3, H3)


def loss_and_grad(p, h, x, t, bf16_storage=False):
    """Mean-squared error over B x 8 outputs and its gradient (flat vector)."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(p, h)
    r = bf16 if bf16_storage else (lambda a: np.asarray(a, np.float64))
    Y, (X, Z1, H1, Z2, H2, Z3, H3) = forward(p, h, x, bf16_storage)
    B = x.shape[0]
    D = Y - t
    loss = float((D * D).mean())
    dY = 2.0 * D / (B * 8)
    dYr = r(dY)
    gW4 = H3.T @ dYr
    gb4 = dY.sum(0)
    dZ3 = (dYr @ r(W4).T) * dgelu(Z3)
    dZ3r = r(dZ3)
    gW3 = H2.T @ dZ3r
    gb3 = dZ3.sum(0)
    dZ2 = (dZ3r @ r(W3).T) * dgelu(Z2)
    dZ2r = r(dZ2)
    gW2 = H1.T @ dZ2r
    gb2 = dZ2.sum(0)
    dZ1 = (dZ2r @ r(W2).T) * dgelu(Z1)
    dZ1r = r(dZ1)
    gW1 = X.T @ dZ1r
    gb1 = dZ1.sum(0)
    return loss, pack([gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4])


QUANT = [0, 1, 4, 5, 6, 8, 11, 3]  # <U>, <V>, <phi>, <uu>, <vv>, <uv>, <phi'^2>, <omega>


def features(mesh, stats):
    """48 features per node: for each of the 8 statistics, the node value, the
    mean, standard deviation, min and max over the node and its neighbours
    (points sharing an element, periodic nodes identified) and the magnitude
    of the average of the element gradients around the node."""
    nn = mesh.n_nodes
    master = mesh.node_master
    en = master[mesh.elem_nodes]
    nbrs = [set() for _ in range(nn)]
    elems = [[] for _ in range(nn)]
    for e in range(mesh.n_elems):
        q = en[e]
        for k in range(3):
            if e not in elems[q[k]]:
                elems[q[k]].append(e)
            for j in range(3):
                if q[j] != q[k]:
                    nbrs[q[k]].add(q[j])
    p = mesh.node_xy[mesh.elem_nodes]
    xBA = p[:, 1, 0] - p[:, 0, 0]
    yBA = p[:, 1, 1] - p[:, 0, 1]
    xCA = p[:, 2, 0] - p[:, 0, 0]
    yCA = p[:, 2, 1] - p[:, 0, 1]
    twoA = xBA * yCA - xCA * yBA
    dNdx = np.stack([(yBA - yCA) / twoA, yCA / twoA, -yBA / twoA], 1)
    dNdy = np.stack([(xCA - xBA) / twoA, -xCA / twoA, xBA / twoA], 1)
    F = np.zeros((nn, 48))
    for n in range(nn):
        q = master[n]
        ring = [q] + sorted(nbrs[q])
        for a, fld in enumerate(QUANT):
            v = stats[fld, ring]
            g = np.zeros(2)
            for e in elems[q]:
                vals = stats[fld, en[e]]
                g += [dNdx[e] @ vals, dNdy[e] @ vals]
            g /= max(1, len(elems[q]))
            F[n, 6 * a:6 * a + 6] = [stats[fld, q], v.mean(), v.std(), v.min(), v.max(), np.hypot(*g)]
    return F
