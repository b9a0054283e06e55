"""AC optimal power flow of the post-contingency main island (Section II.B.1).

The paper runs an AC OPF per scenario and calls the scenario severe when the
OPF does not converge or the converged point violates operating limits; it
does not say which solver.  This oracle uses a primal-dual interior-point
method with one dense KKT solve per Newton step:

  minimise   f(x) = sum_g c2 (Sb Pg)^2 + c1 Sb Pg + c0
  subject to g(x) = 0  (P and Q balance at every island bus)
             h(x) <= 0 (|Sf|^2, |St|^2 <= rate^2 for rated branches, then the
                        V, Pg, Qg boxes as lower/upper pairs)
  variables  x = [theta (island buses, reference removed), V, Pg, Qg]

Newton step on the barrier KKT conditions, reduced to
  [ M   Jg^T ] [dx]   [ -N ]      M = Hess L + Jh^T diag(mu/z) Jh
  [ Jg   0   ] [dl] = [ -g ],     N = grad L + Jh^T Z^-1 (gamma e + mu*h)
then dz = -h - z - Jh dx, dmu = -mu + Z^-1 (gamma e - mu*dz), fraction-to-
boundary step lengths (xi = 0.99995), barrier gamma = sigma z'mu / n_ineq with
sigma = 0.1; a barrier above ``gamma_max`` means divergence.  Start:
theta = 0, V = clip(1), Pg, Qg at box midpoints, z = max(-h, 1), gamma = 1,
mu = gamma / z, lambda = 0.  Converged when the
feasibility, gradient, complementarity and cost-change measures are all
below ``tol``.

Derivatives of the complex power S_k = V_k conj(sum_m M_km V_m) in polar
coordinates, with W_km = V_rk conj(M_km) conj(V_m) (r_k the bus multiplying
row k):
  dS/dtheta = j (diag(S) C - W),  dS/dV = (diag(S) C + W) diag(1/V)
and for a weighted form F = sum_km c_km V_k conj(V_m), T = diag(V) c diag(conj V),
rs/cs its row/column sums:
  F_tt = -diag(rs + cs) + T + T^T
  F_tv[a,b] = j/V_b (delta_ab (rs_a - cs_a) + T_ab - T_ba)
  F_vv[a,b] = (T_ab + T_ba) / (V_a V_b)
(real parts taken for the Lagrangian).
"""
from __future__ import annotations

import dataclasses
import numpy as np
import scipy.linalg as sla

CONVERGED, MAXIT, NUMERICAL, NOT_RUN = 0, 1, 2, 3


@dataclasses.dataclass
class OPFOptions:
    tol: float = 1e-8
    max_it: int = 150
    xi: float = 0.99995
    sigma: float = 0.1
    gamma_max: float = 1e10     # barrier blow-up => diverged (NUMERICAL)
    # Rounding probes, for the tests only (the method's solve is the dense LU,
    # the default): "qr" solves each Newton system by Householder QR instead;
    # row_scale_seed multiplies the rows of each system by powers of two drawn
    # from that seed before the LU.  Both are exact reformulations of the same
    # step, so a scenario whose outcome changes under them is decided by
    # rounding, not by the method.
    kkt_solve: str = "lu"
    row_scale_seed: int | None = None
    # perm_seed: solve each system with its unknowns and equations permuted
    # by one random permutation drawn from that seed (P K P^T) (P d) = P rhs,
    # which changes the elimination order
    perm_seed: int | None = None


@dataclasses.dataclass
class OPFResult:
    status: int
    iters: int
    cost: float
    vm: np.ndarray
    va: np.ndarray
    pg: np.ndarray
    qg: np.ndarray
    lam: np.ndarray
    mu: np.ndarray
    z: np.ndarray
    metrics: tuple          # (feas, grad, comp, dcost) at exit
    max_violation: float
    history: list = dataclasses.field(default_factory=list)


def complex_power_jac(M, rowbus, V):
    """S = V[rowbus] * conj(M @ V) and its polar Jacobians (dense)."""
    S = V[rowbus] * np.conj(M @ V)
    W = V[rowbus][:, None] * np.conj(M) * np.conj(V)[None, :]
    C = np.zeros(M.shape)
    C[np.arange(M.shape[0]), rowbus] = 1.0
    dth = 1j * (S[:, None] * C - W)
    dvm = (S[:, None] * C + W) / np.abs(V)[None, :]
    return S, dth, dvm


def weighted_hessian(c, V):
    """Real parts of the second derivatives of F = sum c_km V_k conj(V_m)
    with respect to (theta, V); returns the full 2n x 2n matrix."""
    vm = np.abs(V)
    T = V[:, None] * c * np.conj(V)[None, :]
    rs, cs = T.sum(axis=1), T.sum(axis=0)
    Htt = -np.diag(rs + cs) + T + T.T
    Htv = 1j * (np.diag(rs - cs) + T - T.T) / vm[None, :]
    Hvv = (T + T.T) / np.outer(vm, vm)
    H = np.block([[Htt, Htv], [Htv.T, Hvv]])
    return H.real


class OPFProblem:
    """Functions of the OPF on one compact island (see module docstring)."""

    def __init__(self, net, sub):
        self.sub = sub
        nb, ng = sub.nb, len(sub.gen)
        self.nb, self.ng = nb, ng
        self.sb = float(net["base_mva"])
        self.c2 = net["c2"][sub.gen]
        self.c1 = net["c1"][sub.gen]
        self.c0 = net["c0"][sub.gen]
        self.pmin, self.pmax = net["pmin"][sub.gen], net["pmax"][sub.gen]
        self.qmin, self.qmax = net["qmin"][sub.gen], net["qmax"][sub.gen]
        self.Cg = np.zeros((nb, ng))
        self.Cg[sub.gbus, np.arange(ng)] = 1.0
        self.rated = np.flatnonzero(sub.rate > 0)
        # variable layout: theta (without ref), V, Pg, Qg
        self.th_cols = np.array([k for k in range(nb) if k != sub.ref], int)
        self.nx = (nb - 1) + nb + 2 * ng
        self.n_ineq = 2 * len(self.rated) + 2 * nb + 4 * ng

    # --- variable packing -------------------------------------------------
    def unpack(self, x):
        nb, ng = self.nb, self.ng
        va = np.zeros(nb)
        va[self.th_cols] = x[:nb - 1]
        vm = x[nb - 1:2 * nb - 1]
        pg = x[2 * nb - 1:2 * nb - 1 + ng]
        qg = x[2 * nb - 1 + ng:]
        return va, vm, pg, qg

    def pack(self, va, vm, pg, qg):
        return np.concatenate([va[self.th_cols], vm, pg, qg])

    def polar_cols(self, D):
        """Drop the reference-angle column of a [d/dtheta, d/dV] block."""
        nb = self.nb
        return np.concatenate([D[:, self.th_cols], D[:, nb:]], axis=1)

    # --- objective --------------------------------------------------------
    def cost(self, x):
        _, _, pg, _ = self.unpack(x)
        p = self.sb * pg
        return float(np.sum(self.c2 * p * p + self.c1 * p + self.c0))

    def cost_grad(self, x):
        _, _, pg, _ = self.unpack(x)
        g = np.zeros(self.nx)
        i0 = 2 * self.nb - 1
        g[i0:i0 + self.ng] = 2 * self.c2 * self.sb ** 2 * pg + self.c1 * self.sb
        return g

    def cost_hess(self):
        H = np.zeros((self.nx, self.nx))
        i0 = 2 * self.nb - 1
        idx = np.arange(i0, i0 + self.ng)
        H[idx, idx] = 2 * self.c2 * self.sb ** 2
        return H

    # --- constraints ------------------------------------------------------
    def evaluate(self, x):
        """g, h, Jg, Jh and the per-block data needed for the Hessian."""
        sub, nb, ng = self.sub, self.nb, self.ng
        va, vm, pg, qg = self.unpack(x)
        V = vm * np.exp(1j * va)
        S, dSth, dSvm = complex_power_jac(sub.Y, np.arange(nb), V)
        g = np.concatenate([S.real + sub.pd - self.Cg @ pg,
                            S.imag + sub.qd - self.Cg @ qg])
        dS = self.polar_cols(np.concatenate([dSth, dSvm], axis=1))
        Jg = np.zeros((2 * nb, self.nx))
        Jg[:nb, :2 * nb - 1] = dS.real
        Jg[nb:, :2 * nb - 1] = dS.imag
        Jg[:nb, 2 * nb - 1:2 * nb - 1 + ng] = -self.Cg
        Jg[nb:, 2 * nb - 1 + ng:] = -self.Cg

        rated = self.rated
        Sf, dSf_th, dSf_vm = complex_power_jac(sub.Yf[rated], sub.f[rated], V)
        St, dSt_th, dSt_vm = complex_power_jac(sub.Yt[rated], sub.t[rated], V)
        dSf = self.polar_cols(np.concatenate([dSf_th, dSf_vm], axis=1))
        dSt = self.polar_cols(np.concatenate([dSt_th, dSt_vm], axis=1))
        rate2 = sub.rate[rated] ** 2
        hf = (Sf * np.conj(Sf)).real - rate2
        ht = (St * np.conj(St)).real - rate2
        nr = len(rated)
        Jh = np.zeros((self.n_ineq, self.nx))
        Jh[:nr, :2 * nb - 1] = 2 * (np.conj(Sf)[:, None] * dSf).real
        Jh[nr:2 * nr, :2 * nb - 1] = 2 * (np.conj(St)[:, None] * dSt).real
        o = 2 * nr
        iv = np.arange(nb)
        Jh[o + iv, nb - 1 + iv] = -1.0
        Jh[o + nb + iv, nb - 1 + iv] = 1.0
        o += 2 * nb
        ig = np.arange(ng)
        Jh[o + ig, 2 * nb - 1 + ig] = -1.0
        Jh[o + ng + ig, 2 * nb - 1 + ig] = 1.0
        o += 2 * ng
        Jh[o + ig, 2 * nb - 1 + ng + ig] = -1.0
        Jh[o + ng + ig, 2 * nb - 1 + ng + ig] = 1.0
        h = np.concatenate([hf, ht, sub.vmin - vm, vm - sub.vmax,
                            self.pmin - pg, pg - self.pmax,
                            self.qmin - qg, qg - self.qmax])
        aux = dict(V=V, Sf=Sf, St=St, dSf=dSf, dSt=dSt, rated=rated)
        return g, h, Jg, Jh, aux

    def lagrangian_hessian(self, x, lam, mu, aux):
        """Hessian of f + lam'g + mu'h with respect to x."""
        sub, nb = self.sub, self.nb
        V = aux["V"]
        H = self.cost_hess()
        # power balance: sum lamP P + lamQ Q = Re(sum (lamP - j lamQ) S)
        c = (lam[:nb] - 1j * lam[nb:])[:, None] * np.conj(sub.Y)
        Hb = weighted_hessian(c, V)
        # flow limits: mu * |S|^2 -> 2 Re(J^T diag(mu) conj J)
        #                            + 2 Re(Hess of sum mu conj(S) S)
        rated = aux["rated"]
        nr = len(rated)
        mf, mt = mu[:nr], mu[nr:2 * nr]
        wf = mf * np.conj(aux["Sf"])
        wt = mt * np.conj(aux["St"])
        Cf = np.zeros((nr, nb))
        Cf[np.arange(nr), sub.f[rated]] = 1.0
        Ct = np.zeros((nr, nb))
        Ct[np.arange(nr), sub.t[rated]] = 1.0
        cflow = (Cf.T @ (wf[:, None] * np.conj(sub.Yf[rated]))
                 + Ct.T @ (wt[:, None] * np.conj(sub.Yt[rated])))
        Hf = 2.0 * weighted_hessian(cflow, V)
        keep = np.concatenate([self.th_cols, nb + np.arange(nb)])
        Hnet = (Hb + Hf)[np.ix_(keep, keep)]
        dSf, dSt = aux["dSf"], aux["dSt"]
        Hnet = Hnet + 2.0 * (dSf.T @ (mf[:, None] * np.conj(dSf))).real
        Hnet = Hnet + 2.0 * (dSt.T @ (mt[:, None] * np.conj(dSt))).real
        H[:2 * nb - 1, :2 * nb - 1] += Hnet
        return H

    def max_violation(self, x, aux):
        sub = self.sub
        va, vm, pg, qg = self.unpack(x)
        v = [vm - sub.vmax, sub.vmin - vm, pg - self.pmax, self.pmin - pg,
             qg - self.qmax, self.qmin - qg]
        if len(aux["rated"]):
            r = sub.rate[aux["rated"]]
            v += [np.abs(aux["Sf"]) - r, np.abs(aux["St"]) - r]
        return float(max(np.max(a) for a in v if len(a)))

    def initial_point(self):
        sub = self.sub
        va = np.zeros(self.nb)
        vm = np.clip(1.0, sub.vmin, sub.vmax)
        pg = 0.5 * (self.pmin + self.pmax)
        qg = 0.5 * (self.qmin + self.qmax)
        return self.pack(va, vm, pg, qg)


def kkt_system(P, x, lam, mu, z, gamma, g, h, Jg, Jh, Lx, aux):
    """The reduced Newton system [M Jg'; Jg 0] [dx; dlam] = [-N; -g]."""
    neq = len(g)
    Hl = P.lagrangian_hessian(x, lam, mu, aux)
    zinv = 1.0 / z
    M = Hl + Jh.T @ ((mu * zinv)[:, None] * Jh)
    N = Lx + Jh.T @ (zinv * (gamma + mu * h))
    K = np.block([[M, Jg.T], [Jg, np.zeros((neq, neq))]])
    rhs = -np.concatenate([N, g])
    return K, rhs


def initial_state(P):
    """Start of the iteration: x0, z0 = max(-h, 1), gamma = 1, mu = 1/z, lam = 0."""
    x = P.initial_point()
    g, h, Jg, Jh, aux = P.evaluate(x)
    z = np.maximum(-h, 1.0)
    gamma = 1.0
    mu = gamma / z
    lam = np.zeros(2 * P.nb)
    return x, lam, z, mu, gamma


def solve_opf(net, sub, opts: OPFOptions = OPFOptions(), keep_history=False) -> OPFResult:
    """Primal-dual interior point, one dense LU-solved KKT system per step."""
    P = OPFProblem(net, sub)
    nx, neq, ni = P.nx, 2 * P.nb, P.n_ineq
    x = P.initial_point()
    g, h, Jg, Jh, aux = P.evaluate(x)
    f = P.cost(x)
    z = np.maximum(-h, 1.0)
    gamma = 1.0
    mu = gamma / z
    lam = np.zeros(neq)
    f_prev = f
    it = 0
    status = MAXIT
    hist = []
    if opts.kkt_solve not in ("lu", "qr"):
        raise ValueError(f"kkt_solve must be 'lu' or 'qr', not {opts.kkt_solve!r}")
    scale_rng = (np.random.default_rng(opts.row_scale_seed)
                 if opts.row_scale_seed is not None else None)
    perm = (np.random.default_rng(opts.perm_seed).permutation(nx + neq)
            if opts.perm_seed is not None else None)
    while True:
        Lx = P.cost_grad(x) + Jg.T @ lam + Jh.T @ mu
        xn = np.max(np.abs(x)) if nx else 0.0
        feas = max(np.max(np.abs(g)), np.max(h)) / (1.0 + max(xn, np.max(np.abs(z))))
        grad = np.max(np.abs(Lx)) / (1.0 + max(np.max(np.abs(lam)), np.max(np.abs(mu))))
        comp = float(z @ mu) / (1.0 + xn)
        dcost = abs(f - f_prev) / (1.0 + abs(f_prev))
        metrics = (feas, grad, comp, dcost)
        if keep_history:
            hist.append(dict(it=it, f=f, metrics=metrics, gamma=gamma))
        if it > 0 and max(metrics) < opts.tol:
            status = CONVERGED
            break
        if it >= opts.max_it:
            status = MAXIT
            break
        it += 1
        K, rhs = kkt_system(P, x, lam, mu, z, gamma, g, h, Jg, Jh, Lx, aux)
        zinv = 1.0 / z
        if not np.all(np.isfinite(K)) or not np.all(np.isfinite(rhs)):
            status = NUMERICAL
            break
        if opts.kkt_solve == "qr":
            q, r = sla.qr(K, check_finite=False)
            if np.any(np.diag(r) == 0.0):
                status = NUMERICAL
                break
            d = sla.solve_triangular(r, q.T @ rhs, check_finite=False)
        else:
            if scale_rng is not None:
                dscale = 2.0 ** scale_rng.integers(-2, 3, K.shape[0])
                K, rhs = dscale[:, None] * K, dscale * rhs
            if perm is not None:
                K, rhs = K[np.ix_(perm, perm)], rhs[perm]
            lu, piv = sla.lu_factor(K, check_finite=False)
            if np.any(np.diag(lu) == 0.0):
                status = NUMERICAL
                break
            d = sla.lu_solve((lu, piv), rhs, check_finite=False)
            if perm is not None:
                d = d[np.argsort(perm)]
        if not np.all(np.isfinite(d)):
            status = NUMERICAL
            break
        dx, dlam = d[:nx], d[nx:]
        dz = -h - z - Jh @ dx
        dmu = -mu + zinv * (gamma - mu * dz)
        neg = dz < 0
        ap = min(opts.xi * np.min(-z[neg] / dz[neg]), 1.0) if np.any(neg) else 1.0
        neg = dmu < 0
        ad = min(opts.xi * np.min(-mu[neg] / dmu[neg]), 1.0) if np.any(neg) else 1.0
        x = x + ap * dx
        z = z + ap * dz
        lam = lam + ad * dlam
        mu = mu + ad * dmu
        if ni:
            gamma = opts.sigma * float(z @ mu) / ni
        if not gamma <= opts.gamma_max:
            status = NUMERICAL
            break
        f_prev = f
        g, h, Jg, Jh, aux = P.evaluate(x)
        f = P.cost(x)
        if not (np.all(np.isfinite(x)) and np.all(np.isfinite(z))
                and np.all(np.isfinite(mu)) and np.all(np.isfinite(lam))):
            status = NUMERICAL
            break
    va, vm, pg, qg = P.unpack(x)
    mv = P.max_violation(x, aux) if status != NUMERICAL else float("nan")
    return OPFResult(status=status, iters=it, cost=f, vm=vm, va=va, pg=pg,
                     qg=qg, lam=lam, mu=mu, z=z, metrics=metrics,
                     max_violation=mv, history=hist)
