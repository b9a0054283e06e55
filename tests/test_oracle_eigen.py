"""Pins for the eigenvalue step (Section II.B.2): matrices with known
spectra, trace and determinant invariants, and the plain Francis QR against
LAPACK."""
import numpy as np
import pytest

from oracle import eigen


def _match(a, b):
    a = sorted(a, key=lambda z: (round(z.real, 9), round(z.imag, 9)))
    b = list(b)
    out = 0.0
    for z in a:
        k = int(np.argmin(np.abs(np.array(b) - z)))
        out = max(out, abs(b[k] - z) / max(1.0, abs(z)))
        b.pop(k)
    return out


def _known(rng, reals, pairs):
    n = len(reals) + 2 * len(pairs)
    B = np.zeros((n, n))
    k = 0
    for r in reals:
        B[k, k] = r
        k += 1
    for s, w in pairs:
        B[k:k + 2, k:k + 2] = [[s, w], [-w, s]]
        k += 2
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = list(reals) + [complex(s, w) for s, w in pairs] + [complex(s, -w) for s, w in pairs]
    return Q @ B @ Q.T, np.array(lam, complex)


@pytest.mark.parametrize("seed", range(3))
def test_known_spectrum(seed):
    rng = np.random.default_rng(seed)
    A, lam = _known(rng, rng.uniform(-5, -0.1, 9), [(-0.3, 7.0), (-0.05, 2.0), (0.2, 11.0)])
    assert _match(eigen.eigvals(A), lam) < 1e-10
    assert _match(eigen.francis_eigvals(A), lam) < 1e-10
    alpha, zeta = eigen.spectral_summary(lam)
    assert alpha == pytest.approx(0.2)
    assert zeta == pytest.approx(-0.2 / abs(complex(0.2, 11.0)))


def test_companion_roots():
    roots = np.array([-1.0, -2.0, -0.5 + 3j, -0.5 - 3j, -4.0])
    c = np.poly(roots).real
    n = len(roots)
    C = np.zeros((n, n))
    C[0, :] = -c[1:]
    C[1:, :-1] = np.eye(n - 1)
    assert _match(eigen.francis_eigvals(C), roots) < 1e-9
    assert _match(eigen.eigvals(C), roots) < 1e-9


@pytest.mark.parametrize("n", [5, 17, 40])
def test_francis_matches_lapack_and_invariants(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    l1 = eigen.francis_eigvals(A)
    l2 = eigen.eigvals(A)
    assert _match(l1, l2) < 1e-9
    assert abs(l1.sum().real - np.trace(A)) < 1e-10 * np.linalg.norm(A)
    sign, logdet = np.linalg.slogdet(A)
    assert abs(np.sum(np.log(np.abs(l1))) - logdet) < 1e-8 * n


def test_hessenberg_is_similarity():
    rng = np.random.default_rng(9)
    A = rng.standard_normal((12, 12))
    H = eigen.hessenberg(A)
    assert np.allclose(np.tril(H, -2), 0)
    assert _match(np.linalg.eigvals(H), np.linalg.eigvals(A)) < 1e-10


def test_summary_without_oscillation():
    assert eigen.spectral_summary(np.array([-1.0, -2.0, 0.0])) == (0.0, 1.0)
