"""Oracle for the learned preconditioner (TEST INFRASTRUCTURE ONLY).

Plain numpy, FP64.  The task adds to the paper's Backward Euler solve
(Sec. 3.1: PCG with the point-Jacobi preconditioner PC1) a small
convolutional network that corrects the Jacobi step inside flexible CG.
Nothing here comes from the paper's text beyond that solve; the network,
its features, the loss and the flexible-CG variant are this project's
reading of the task:

* network N: three 3x3x3 convolutions 8 -> 16 (+bias, ReLU) -> 16 (+bias,
  ReLU) -> 1 (no bias) on the cell grid, zero padding in r and theta,
  periodic in phi;
* preconditioner P(r) = r/D + sigma N(c) with D the Jacobi diagonal,
  sigma = RMS(r/D), input channels c0 = (r/D)/sigma, c1 = V/D and
  c2..c7 = -M_{m,nb}/D_m for the six face neighbours (r-, r+, t-, t+, p-,
  p+; zero where the neighbour does not exist).  P is positively
  homogeneous: P(a r) = a P(r) for a > 0;
* loss per (residual r, error e) pair, in the energy norm of the system
  matrix M that CG minimises: |P(r) - e|_M^2 / |e|_M^2;
* flexible CG truncated to one previous direction (Notay 2000):
  beta = -<z, q_prev>/<p_prev, q_prev>, alpha = <p, r>/<p, q>.

Numerics of the GPU network: BF16 (round to nearest even) weights, inputs
and stored activations, FP32 accumulation, bias and ReLU.  `forward(...,
bf16=True)` emulates the roundings (accumulating in FP64).
"""
from __future__ import annotations

import numpy as np

CIN = (8, 16, 16)
COUT = (16, 16, 1)
NPARAM = sum(co * ci * 27 for ci, co in zip(CIN, COUT)) + COUT[0] + COUT[1]


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    rnd = ((b >> 16) & 1) + 0x7FFF
    out = ((b + rnd) >> 16) << 16
    out = out.astype(np.uint32).view(np.float32)
    # NaN/Inf pass through unchanged
    out = np.where(np.isfinite(f), out, f)
    return out.astype(np.float64)


def unpack(theta):
    """Flat parameter vector -> [W1, b1, W2, b2, W3] (W: [co, ci, 3, 3, 3])."""
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for layer, (ci, co) in enumerate(zip(CIN, COUT)):
        n = co * ci * 27
        out.append(theta[o:o + n].reshape(co, ci, 3, 3, 3))
        o += n
        if layer < 2:
            out.append(theta[o:o + co])
            o += co
    assert o == NPARAM
    return out


def pack(params):
    return np.concatenate([p.ravel() for p in params])


def he_init(rng):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases."""
    ps = []
    for layer, (ci, co) in enumerate(zip(CIN, COUT)):
        ps.append(rng.standard_normal((co, ci, 3, 3, 3)) * np.sqrt(2.0 / (ci * 27)))
        if layer < 2:
            ps.append(np.zeros(co))
    return pack(ps)


def _shift(x, di, dj, dk, periodic=True):
    """y[.., i, j, k] = x[.., i+di, j+dj, (k+dk) mod np], zero outside r, theta
    (and outside phi when not periodic)."""
    y = np.roll(x, -dk, axis=-1)
    if not periodic and dk != 0:
        y = y.copy()
        if dk > 0:
            y[..., -dk:] = 0.0
        else:
            y[..., :-dk] = 0.0
    nr, nt = x.shape[-3], x.shape[-2]
    out = np.zeros_like(y)
    ri = slice(max(0, -di), min(nr, nr - di))
    ro = slice(max(0, di), min(nr, nr + di))
    tj = slice(max(0, -dj), min(nt, nt - dj))
    to = slice(max(0, dj), min(nt, nt + dj))
    out[..., ri, tj, :] = y[..., ro, to, :]
    return out


def conv(W, x, periodic=True):
    """3x3x3 convolution (cross-correlation) of x [ci, nr, nt, np]."""
    co = W.shape[0]
    y = np.zeros((co,) + x.shape[1:])
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for dk in (-1, 0, 1):
                xs = _shift(x, di, dj, dk, periodic)
                y += np.einsum("oc,c...->o...", W[:, :, di + 1, dj + 1, dk + 1], xs)
    return y


def conv_t(W, g, periodic=True):
    """Adjoint of conv in its input: x-gradient for output-gradient g."""
    ci = W.shape[1]
    x = np.zeros((ci,) + g.shape[1:])
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for dk in (-1, 0, 1):
                t = np.einsum("oc,o...->c...", W[:, :, di + 1, dj + 1, dk + 1], g)
                x += _shift(t, -di, -dj, -dk, periodic)
    return x


def conv_wgrad(x, g, periodic=True):
    """dW[co, ci, tap] = sum_points g[co, p] x[ci, p + tap]."""
    co, ci = g.shape[0], x.shape[0]
    dW = np.zeros((co, ci, 3, 3, 3))
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for dk in (-1, 0, 1):
                xs = _shift(x, di, dj, dk, periodic)
                dW[:, :, di + 1, dj + 1, dk + 1] = g.reshape(co, -1) @ xs.reshape(ci, -1).T
    return dW


def forward(theta, c, bf16_mode=False, keep=False, periodic=True):
    """N(c) for input channels c [8, nr, nt, np]; returns [nr, nt, np]."""
    W1, b1, W2, b2, W3 = unpack(theta)
    rd = bf16 if bf16_mode else (lambda v: v)
    x0 = rd(c)
    z1 = conv(rd(W1), x0, periodic) + b1[:, None, None, None]
    a1 = rd(np.maximum(z1, 0.0))
    z2 = conv(rd(W2), a1, periodic) + b2[:, None, None, None]
    a2 = rd(np.maximum(z2, 0.0))
    out = conv(rd(W3), a2, periodic)[0]
    if keep:
        return out, (x0, z1, a1, z2, a2)
    return out


def backward(theta, cache, gout, bf16_mode=False, periodic=True):
    """Gradient of sum(gout * N(c)) with respect to the flat parameters.
    bf16_mode rounds the weights and the stored gradients of the output and
    of each activation to BF16 (the network's storage precision)."""
    W1, b1, W2, b2, W3 = unpack(theta)
    rd = bf16 if bf16_mode else (lambda v: v)
    x0, z1, a1, z2, a2 = cache
    g3 = rd(gout)[None]
    dW3 = conv_wgrad(a2, g3, periodic)
    ga2 = conv_t(rd(W3), g3, periodic)
    gz2 = rd(ga2 * (z2 > 0))
    dW2 = conv_wgrad(a1, gz2, periodic)
    db2 = gz2.sum(axis=(1, 2, 3))
    ga1 = conv_t(rd(W2), gz2, periodic)
    gz1 = rd(ga1 * (z1 > 0))
    dW1 = conv_wgrad(x0, gz1, periodic)
    db1 = gz1.sum(axis=(1, 2, 3))
    return pack([dW1, db1, dW2, db2, dW3])


def features(r, D, V, cpl, dt):
    """Input channels [8, nr, nt, np] for residual r: c0 = (r/D)/sigma,
    c1 = V/D, c2..c7 = -dt cpl[q]/D with cpl the six face couplings."""
    zj = r / D
    sigma = np.sqrt(np.mean(zj * zj))
    c0 = zj / sigma if sigma > 0 else np.zeros_like(zj)
    return np.concatenate([c0[None], (V / D)[None], -dt * cpl / D[None]], axis=0)


def face_couplings(apply_lin, V):
    """cpl[q][m] = L(m, nb_q(m)) for the face neighbours nb = r-, r+, t-, t+,
    p-, p+ (0 where none), read column by column from L x = -V F_lin(x):
    brute force over unit vectors (small grids only)."""
    nr, nt, npp = V.shape
    cpl = np.zeros((6,) + V.shape)
    e = np.zeros(V.shape)
    for i in range(nr):
        for j in range(nt):
            for k in range(npp):
                e[i, j, k] = 1.0
                col = -V * apply_lin(e)          # column n = (i, j, k) of L
                e[i, j, k] = 0.0
                # cells m whose neighbour in direction q is n
                if i + 1 < nr:
                    cpl[0, i + 1, j, k] = col[i + 1, j, k]    # m = n + r: its r- is n
                if i - 1 >= 0:
                    cpl[1, i - 1, j, k] = col[i - 1, j, k]
                if j + 1 < nt:
                    cpl[2, i, j + 1, k] = col[i, j + 1, k]
                if j - 1 >= 0:
                    cpl[3, i, j - 1, k] = col[i, j - 1, k]
                cpl[4, i, j, (k + 1) % npp] = col[i, j, (k + 1) % npp]
                cpl[5, i, j, (k - 1) % npp] = col[i, j, (k - 1) % npp]
    return cpl


def precondition(theta, r, D, static, bf16_mode=False):
    """P(r) = r/D + sigma N(c) on one component r [nr, nt, np]; static
    holds channels c1..c7 [7, nr, nt, np].  theta None: Jacobi only."""
    zj = r / D
    if theta is None:
        return zj
    sigma = np.sqrt(np.mean(zj * zj))
    if sigma == 0.0:
        return zj
    c = np.concatenate([(zj / sigma)[None], static], axis=0)
    return zj + sigma * forward(theta, c, bf16_mode)


def loss_and_grad(theta, pairs, D, static, matvec, bf16_mode=False):
    """Mean over pairs (r, e) of the energy-norm loss
    |P(r) - e|_M^2 / |e|_M^2 (|v|_M^2 = <v, M v>, matvec(v) = M v) and its
    gradient in theta (FP64; bf16_mode emulates the network's roundings)."""
    rd = bf16 if bf16_mode else (lambda v: v)
    L = 0.0
    g = np.zeros(NPARAM)
    n = len(pairs)
    for r, e in pairs:
        zj = r / D
        sigma = np.sqrt(np.mean(zj * zj))
        c = np.concatenate([(zj / sigma)[None], static], axis=0)
        if bf16_mode:
            c = rd(c)
        out, cache = forward(theta, c, bf16_mode, keep=True)
        d = zj + sigma * out - e
        Md = matvec(d)
        den = np.vdot(e, matvec(e))
        L += np.vdot(d, Md) / den
        # d/d(out) of <d, M d> = 2 sigma M d (M symmetric)
        gout = 2.0 * sigma * Md / (den * n)
        g += backward(theta, cache, gout, bf16_mode)
    return L / n, g


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) on FP64 copies; t counts from 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def fcg(matvec, b, x0, D, prec, tol=1e-10, max_iter=10000):
    """Flexible CG truncated to one direction with preconditioner prec(r)
    (Notay 2000); stops when ||r|| <= tol ||b||.  Returns (x, iterations)."""
    x = x0.copy()
    r = b - matvec(x)
    bn = np.linalg.norm(b)
    if np.linalg.norm(r) <= tol * bn:
        return x, 0
    z = prec(r)
    p = z.copy()
    for it in range(1, max_iter + 1):
        q = matvec(p)
        pq = np.vdot(p, q)
        alpha = np.vdot(p, r) / pq
        x += alpha * p
        r -= alpha * q
        if np.linalg.norm(r) <= tol * bn:
            return x, it
        z = prec(r)
        beta = -np.vdot(z, q) / pq
        p = z + beta * p
    return x, max_iter
