"""Eigenvalues of the state matrix and the small-signal test (Section II.B.2).

A scenario is small-signal unstable when some eigenvalue has a non-negative
real part (the paper's "Ri(lambda) >= 0" is read as Re(lambda) >= 0).  The
minimum damping ratio over oscillatory modes is reported beside it.

``eigvals`` is LAPACK's dense nonsymmetric eigensolver (Hessenberg reduction
plus Francis QR) through NumPy.  ``francis_eigvals`` is an independent plain
implementation of the same textbook method (Householder reduction to upper
Hessenberg form, then implicit double-shift QR sweeps with deflation, after
Golub and Van Loan, Matrix Computations, Sections 7.4-7.5), used to cross-check
LAPACK on small matrices.
"""
from __future__ import annotations

import numpy as np

OSC_REL = 1e-8     # |Im| > OSC_REL * |lambda| marks an oscillatory mode


def eigvals(A):
    return np.linalg.eigvals(A)


def spectral_summary(lam):
    """(max real part, minimum damping ratio over oscillatory modes).

    The damping ratio of lambda = s + j w is -s / |lambda|; with no
    oscillatory mode the minimum is reported as 1.0."""
    lam = np.asarray(lam)
    alpha = float(np.max(lam.real)) if lam.size else float("-inf")
    mag = np.abs(lam)
    osc = np.abs(lam.imag) > OSC_REL * mag
    if np.any(osc):
        zeta = float(np.min(-lam.real[osc] / mag[osc]))
    else:
        zeta = 1.0
    return alpha, zeta


# --- plain Hessenberg + Francis double-shift QR ---------------------------

def hessenberg(A):
    """Householder reduction to upper Hessenberg form (similarity)."""
    H = np.array(A, dtype=float, copy=True)
    n = H.shape[0]
    for k in range(n - 2):
        x = H[k + 1:, k].copy()
        alpha = np.linalg.norm(x)
        if alpha == 0.0:
            continue
        v = x
        v[0] += np.copysign(alpha, x[0])
        v /= np.linalg.norm(v)
        H[k + 1:, k:] -= 2.0 * np.outer(v, v @ H[k + 1:, k:])
        H[:, k + 1:] -= 2.0 * np.outer(H[:, k + 1:] @ v, v)
        H[k + 2:, k] = 0.0
    return H


def _eig2(a, b, c, d):
    """Eigenvalues of [[a, b], [c, d]] from the characteristic polynomial."""
    tr = 0.5 * (a + d)
    det = (a - tr) * (d - tr) - b * c
    disc = -det
    if disc >= 0.0:
        s = np.sqrt(disc)
        # avoid cancellation: larger root first, smaller from the product
        r1 = tr + np.copysign(s, tr) if tr != 0.0 else s
        r2 = (a * d - b * c) / r1 if r1 != 0.0 else tr - s
        return complex(r1), complex(r2)
    s = np.sqrt(-disc)
    return complex(tr, s), complex(tr, -s)


def francis_eigvals(A, max_sweeps_per_eig=60):
    """All eigenvalues by implicit double-shift QR on the Hessenberg form."""
    H = hessenberg(A)
    n = H.shape[0]
    out = []
    hi = n - 1
    it = 0
    eps = np.finfo(float).eps
    while hi >= 0:
        if hi == 0:
            out.append(complex(H[0, 0]))
            hi -= 1
            continue
        # find the start of the unreduced block ending at hi
        lo = hi
        while lo > 0:
            s = abs(H[lo - 1, lo - 1]) + abs(H[lo, lo])
            if s == 0.0:
                s = np.abs(H[:hi + 1, :hi + 1]).sum()
            if abs(H[lo, lo - 1]) <= eps * s:
                H[lo, lo - 1] = 0.0
                break
            lo -= 1
        if lo == hi:
            out.append(complex(H[hi, hi]))
            hi -= 1
            it = 0
            continue
        if lo == hi - 1:
            out.extend(_eig2(H[hi - 1, hi - 1], H[hi - 1, hi],
                             H[hi, hi - 1], H[hi, hi]))
            hi -= 2
            it = 0
            continue
        it += 1
        if it > max_sweeps_per_eig:
            raise np.linalg.LinAlgError("QR did not converge")
        # shifts: eigenvalues of the trailing 2x2 (exceptional every 10)
        if it % 10 == 0:
            w = abs(H[hi, hi - 1]) + abs(H[hi - 1, hi - 2])
            s_sum, s_prod = 1.5 * w, w * w
        else:
            a, b = H[hi - 1, hi - 1], H[hi - 1, hi]
            c, d = H[hi, hi - 1], H[hi, hi]
            s_sum, s_prod = a + d, a * d - b * c
        # first column of (H - s1)(H - s2) restricted to the block
        h = H
        x = h[lo, lo] * h[lo, lo] + h[lo, lo + 1] * h[lo + 1, lo] \
            - s_sum * h[lo, lo] + s_prod
        y = h[lo + 1, lo] * (h[lo, lo] + h[lo + 1, lo + 1] - s_sum)
        z = h[lo + 1, lo] * h[lo + 2, lo + 1]
        for k in range(lo, hi - 1):
            v = np.array([x, y, z])
            nv = np.linalg.norm(v)
            if nv != 0.0:
                v[0] += np.copysign(nv, v[0])
                v /= np.linalg.norm(v)
                c0 = max(lo, k - 1)
                H[k:k + 3, c0:hi + 1] -= 2.0 * np.outer(v, v @ H[k:k + 3, c0:hi + 1])
                r1 = min(k + 3, hi)
                H[lo:r1 + 1, k:k + 3] -= 2.0 * np.outer(H[lo:r1 + 1, k:k + 3] @ v, v)
            x = H[k + 1, k]
            y = H[k + 2, k]
            if k < hi - 2:
                z = H[k + 3, k]
        v = np.array([x, y])
        nv = np.linalg.norm(v)
        if nv != 0.0:
            v[0] += np.copysign(nv, v[0])
            v /= np.linalg.norm(v)
            H[hi - 1:hi + 1, hi - 2:hi + 1] -= 2.0 * np.outer(v, v @ H[hi - 1:hi + 1, hi - 2:hi + 1])
            H[lo:hi + 1, hi - 1:hi + 1] -= 2.0 * np.outer(H[lo:hi + 1, hi - 1:hi + 1] @ v, v)
    return np.array(out)
