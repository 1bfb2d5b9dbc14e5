"""Oracle of the feature-pass adjoint -- TEST INFRASTRUCTURE ONLY (same rules as the package).

Reverse mode of the feature pass: given dL/d(g, k, V, gmax) it returns dL/dI, so a loss on the
rendered image reaches the intensities through the morphology terms of Eq. 4 as well as through
the TF lookup.  Plain NumPy in FP64, written with explicit per-axis matrices so that every linear
step is a matrix and its adjoint is that matrix's transpose:

  D1_a  clamped central difference along axis a, (I[i+1] - I[i-1]) / (2 h_a)   Sec. 2.3 Eq. 2
  D2_a  clamped second difference, (s[i+1] - 2 s[i] + s[i-1]) / h_a^2
  G_a   clamped, sampled, normalized Gaussian of radius floor(3 sigma/h_a + 1/2)  (Hessian scale)

  g_a = D1_a I                                      (Eq. 2)
  H_aa = D2_a S,  H_ab = D1_a D1_b S,  S = G_x G_y G_z I   (per scale; Sec. 1 and 2.3)
  k = g^T H_0 g / g^T g  (0 where g = 0)            (Eq. 3, first scale)
  V = max over scales of Frangi(eig(sigma^2 H))     (Sec. 1; the first scale reaching the maximum
                                                     strictly above 0 is the one differentiated)
  gmax = max |g|                                    (Eq. 4's normalizer; the first voxel in index
                                                     order attaining it is the one differentiated)

Local derivatives: dk/dg = 2 (H g - k g) / g^T g, dk/dH_ab = g_a g_b / g^T g (times 2 for a != b,
the entry standing for both (a, b) and (b, a)); dV/dA = sum_i dV/dlambda_i e_i e_i^T for the
eigenpairs (lambda_i, e_i) of A = sigma^2 H (numpy.linalg.eigh), sorted by (|lambda|, lambda) as
the forward sorts them; the Frangi partials are differentiated term by term.  At V = 0 (lambda2 >= 0
or lambda3 >= 0), k at g = 0 and the eigenvalue crossings the derivative is taken as 0 / is undefined
(measure-zero sets).  Frangi's c must be given (> 0).

The forward in this matrix form (``forward``) is pinned against the loop-form C oracle, and the
adjoint against FP64 central differences of the C oracle's forward, in tests/test_oracle_grad.py.
"""
from __future__ import annotations

import numpy as np

AX = {0: 2, 1: 1, 2: 0}  # axis a (x, y, z) -> numpy axis of a [nz][ny][nx] array
PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))  # order xx, yy, zz, xy, xz, yz


def gauss_matrix(n, sigma_vox):
    r = max(int(np.floor(3.0 * sigma_vox + 0.5)), 1)
    t = np.arange(-r, r + 1)
    w = np.exp(-(t * t) / (2.0 * sigma_vox * sigma_vox))
    w /= w.sum()
    G = np.zeros((n, n))
    for i in range(n):
        for k, wk in zip(t, w):
            G[i, min(max(i + k, 0), n - 1)] += wk
    return G


def d1_matrix(n, h):
    D = np.zeros((n, n))
    for i in range(n):
        D[i, min(i + 1, n - 1)] += 1.0 / (2.0 * h)
        D[i, max(i - 1, 0)] -= 1.0 / (2.0 * h)
    return D


def d2_matrix(n, h):
    D = np.zeros((n, n))
    for i in range(n):
        D[i, min(i + 1, n - 1)] += 1.0 / (h * h)
        D[i, i] -= 2.0 / (h * h)
        D[i, max(i - 1, 0)] += 1.0 / (h * h)
    return D


def apply(M, vol, a):
    """M (n x n) applied along axis a (0 = x, 1 = y, 2 = z) of a [nz][ny][nx] array."""
    ax = AX[a]
    return np.moveaxis(np.tensordot(M, vol, axes=(1, ax)), 0, ax)


def _shape_n(shape):
    return (shape[2], shape[1], shape[0])  # (nx, ny, nz)


def scale_operators(shape, spacing, sigma_mm):
    """Per axis (G, D1 G, D2 G): the three smoothing-and-difference matrices of one scale."""
    n = _shape_n(shape)
    ops = []
    for a in range(3):
        G = gauss_matrix(n[a], sigma_mm / spacing[a])
        ops.append((G, d1_matrix(n[a], spacing[a]) @ G, d2_matrix(n[a], spacing[a]) @ G))
    return ops


def _filters(a, b):
    """Which operator (0 = G, 1 = D1 G, 2 = D2 G) H_ab applies along each axis."""
    f = [0, 0, 0]
    if a == b:
        f[a] = 2
    else:
        f[a] = 1
        f[b] = 1
    return f


def hessian(I, spacing, sigma_mm, ops=None):
    ops = ops or scale_operators(I.shape, spacing, sigma_mm)
    H = np.empty((6,) + I.shape)
    for e, (a, b) in enumerate(PAIRS):
        f = _filters(a, b)
        x = I
        for ax in range(3):
            x = apply(ops[ax][f[ax]], x, ax)
        H[e] = x
    return H


def hessian_T(Hb, spacing, sigma_mm, ops=None):
    """Adjoint of hessian: sum over the six entries of (their operator)^T applied to Hb[e]."""
    shape = Hb.shape[1:]
    ops = ops or scale_operators(shape, spacing, sigma_mm)
    out = np.zeros(shape)
    for e, (a, b) in enumerate(PAIRS):
        f = _filters(a, b)
        x = Hb[e]
        for ax in range(3):
            x = apply(ops[ax][f[ax]].T, x, ax)
        out += x
    return out


def gradient(I, spacing):
    """Eq. 2 as the difference quotient of the clamped neighbours (the same linear map as D1_a, but
    exactly 0 where the two neighbours are equal, which R5's k = 0 at g = 0 relies on; a matrix
    product can leave a rounding residual there)."""
    g = []
    for a in range(3):
        ax = AX[a]
        n = I.shape[ax]
        idx = np.arange(n)
        up = np.take(I, np.minimum(idx + 1, n - 1), axis=ax)
        dn = np.take(I, np.maximum(idx - 1, 0), axis=ax)
        g.append((up - dn) / (2.0 * spacing[a]))
    return np.stack(g)


def gradient_T(gb, spacing):
    n = _shape_n(gb.shape[1:])
    return sum(apply(d1_matrix(n[a], spacing[a]).T, gb[a], a) for a in range(3))


def _sym(H6):
    """[6][...] -> [...][3][3]."""
    xx, yy, zz, xy, xz, yz = H6
    return np.stack([np.stack([xx, xy, xz], -1), np.stack([xy, yy, yz], -1), np.stack([xz, yz, zz], -1)], -2)


def eig_sorted(A6):
    """Eigenvalues [..., 3] sorted by (|l|, l) and their unit eigenvectors [..., 3 (comp), 3 (i)]."""
    lam, vec = np.linalg.eigh(_sym(A6))
    # stable order by (|l|, l): sort by l first, then stably by |l|
    o1 = np.argsort(lam, axis=-1, kind="stable")
    lam1 = np.take_along_axis(lam, o1, -1)
    o2 = np.argsort(np.abs(lam1), axis=-1, kind="stable")
    order = np.take_along_axis(o1, o2, -1)
    lam = np.take_along_axis(lam, order, -1)
    vec = np.take_along_axis(vec, order[..., None, :], -1)
    return lam, vec


def frangi(lam, alpha, beta, c):
    l1, l2, l3 = lam[..., 0], lam[..., 1], lam[..., 2]
    ok = (l2 < 0) & (l3 < 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        Ra2 = l2 * l2 / (l3 * l3)
        Rb2 = l1 * l1 / np.abs(l2 * l3)
        S2 = l1 * l1 + l2 * l2 + l3 * l3
        V = (1 - np.exp(-Ra2 / (2 * alpha ** 2))) * np.exp(-Rb2 / (2 * beta ** 2)) * (1 - np.exp(-S2 / (2 * c * c)))
    return np.where(ok, V, 0.0)


def frangi_grad(lam, alpha, beta, c):
    """dV/dlambda_i [..., 3] (0 where V = 0 by the sign rule)."""
    l1, l2, l3 = lam[..., 0], lam[..., 1], lam[..., 2]
    ok = (l2 < 0) & (l3 < 0)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        p = l2 * l3  # > 0 where ok
        Ra2 = l2 * l2 / (l3 * l3)
        Rb2 = l1 * l1 / p
        S2 = l1 * l1 + l2 * l2 + l3 * l3
        ea = np.exp(-Ra2 / (2 * alpha ** 2))
        Fa = 1 - ea
        Fb = np.exp(-Rb2 / (2 * beta ** 2))
        ec = np.exp(-S2 / (2 * c * c))
        Fc = 1 - ec
        dFa = ea / (2 * alpha ** 2)          # dFa / dRa2
        dFb = -Fb / (2 * beta ** 2)          # dFb / dRb2
        dFc = ec / (2 * c * c)               # dFc / dS2
        dRa2 = np.stack([np.zeros_like(l1), 2 * l2 / (l3 * l3), -2 * l2 * l2 / (l3 ** 3)], -1)
        dRb2 = np.stack([2 * l1 / p, -l1 * l1 / (l2 * l2 * l3), -l1 * l1 / (l2 * l3 * l3)], -1)
        dS2 = 2 * lam
        G = ((Fb * Fc * dFa)[..., None] * dRa2 + (Fa * Fc * dFb)[..., None] * dRb2
             + (Fa * Fb * dFc)[..., None] * dS2)
    return np.where(ok[..., None], G, 0.0)


def _to6(P):
    """Symmetric [...][3][3] -> the six stored entries' adjoint (diagonal once, off-diagonal twice)."""
    return np.stack([P[..., 0, 0], P[..., 1, 1], P[..., 2, 2], 2 * P[..., 0, 1], 2 * P[..., 0, 2], 2 * P[..., 1, 2]])


def forward(I, spacing, sigmas, alpha=0.5, beta=0.5, c=0.1):
    """The feature pass in matrix form: dict(g, kappa, V, gmax, argmax, H [S][6], win, Vs)."""
    I = np.asarray(I, np.float64)
    g = gradient(I, spacing)
    gn = np.sqrt((g * g).sum(0))
    am = int(np.argmax(gn))  # first occurrence
    Hs, Vs = [], []
    for sg in sigmas:
        H = hessian(I, spacing, sg)
        lam, _ = eig_sorted(sg * sg * H)
        Hs.append(H)
        Vs.append(frangi(lam, alpha, beta, c))
    V = np.zeros(I.shape)
    win = np.full(I.shape, -1)
    for s, vs in enumerate(Vs):
        up = vs > V
        V = np.where(up, vs, V)
        win = np.where(up, s, win)
    H0 = Hs[0]
    gg = (g * g).sum(0)
    with np.errstate(invalid="ignore", divide="ignore"):
        num = sum((1 if a == b else 2) * H0[e] * g[a] * g[b] for e, (a, b) in enumerate(PAIRS))
        kappa = np.where(gg > 0, num / gg, 0.0)
    return dict(g=g, kappa=kappa, V=V, gmax=float(gn.ravel()[am]), argmax=am, H=Hs, win=win, Vs=np.stack(Vs))


def local_adjoint(I, spacing, sigmas, alpha, beta, c, dg, dkappa, dV, dgmax, fw=None):
    """The per-voxel part: returns (dg_total [3][...] to go through D1^T, Hb [S][6][...] to go
    through the Hessian operators' transposes)."""
    assert c > 0, "the adjoint takes Frangi's c as given"
    fw = fw or forward(I, spacing, sigmas, alpha, beta, c)
    g, H0 = fw["g"], fw["H"][0]
    gg = (g * g).sum(0)
    nz = gg > 0
    safe = np.where(nz, gg, 1.0)
    dg_t = np.array(dg, np.float64, copy=True)
    Hg = np.stack([sum(H0[PAIRS.index(tuple(sorted((a, b))))] * g[b] for b in range(3)) for a in range(3)])
    k = fw["kappa"]
    dg_t += np.where(nz, dkappa * 2.0 * (Hg - k * g) / safe, 0.0)
    Hb = np.zeros((len(sigmas), 6) + I.shape)
    for e, (a, b) in enumerate(PAIRS):
        Hb[0, e] = np.where(nz, dkappa * (1 if a == b else 2) * g[a] * g[b] / safe, 0.0)
    for s, sg in enumerate(sigmas):
        lam, vec = eig_sorted(sg * sg * fw["H"][s])
        f = frangi_grad(lam, alpha, beta, c)  # [..., 3]
        P = np.einsum("...i,...ai,...bi->...ab", f, vec, vec)  # sum_i f_i e_i e_i^T
        sel = (fw["win"] == s) * np.asarray(dV, np.float64)
        Hb[s] += sel * sg * sg * _to6(P)
    gn = np.sqrt(gg)
    if fw["gmax"] > 0 and dgmax != 0.0:
        idx = np.unravel_index(fw["argmax"], I.shape)
        for a in range(3):
            dg_t[(a,) + idx] += dgmax * g[(a,) + idx] / gn[idx]
    return dg_t, Hb


def vjp(I, spacing, sigmas, alpha, beta, c, dg, dkappa, dV, dgmax):
    """dL/dI of the feature pass for upstream dL/d(g [3][...], kappa, V, gmax)."""
    I = np.asarray(I, np.float64)
    dg_t, Hb = local_adjoint(I, spacing, sigmas, alpha, beta, c, dg, dkappa, dV, dgmax)
    out = gradient_T(dg_t, spacing)
    for s, sg in enumerate(sigmas):
        out += hessian_T(Hb[s], spacing, sg)
    return out
