// AC OPF of the post-contingency main island (Section II.B.1) by a
// primal-dual interior-point method with one dense KKT solve per Newton step.
//
//   minimise  sum c2 (Sb Pg)^2 + c1 Sb Pg + c0
//   s.t.      P/Q balance at every island bus (g = 0)
//             |Sf|^2, |St|^2 <= rate^2, V, Pg, Qg boxes (h <= 0)
//   Newton:   [M Jg'; Jg 0][dx; dl] = [-N; -g]
//             M = Hess L + Jh' diag(mu/z) Jh,  N = grad L + Jh' (gamma + mu h)/z
//             dz = -h - z - Jh dx,  dmu = -mu + (gamma - mu dz)/z
//   steps:    fraction to the boundary (xi = 0.99995), gamma = 0.1 z'mu/n_ineq
//   start:    theta = 0, V = clip(1), Pg, Qg mid-box, z = max(-h, 1), mu = 1/z
//   stop:     feasibility, gradient, complementarity and cost change < tol;
//             iteration cap; non-finite or exactly singular KKT, or a barrier
//             above gamma_max, is a numerical failure.
//
// One workgroup per scenario.  Branch terms are computed one thread per
// branch into LDS (powers at both ends, their gradients, the 4x4 Lagrangian
// Hessian block over (theta_f, theta_t, V_f, V_t)); bus rows are then gathered
// one thread per bus over its incident branches in a fixed order, so every
// KKT entry has exactly one writer and the result is deterministic.
#include "cs_internal.h"
#include "branch_math.h"

namespace cs {

constexpr int OPF_THREADS = 256;
constexpr double XI = 0.99995;
constexpr double SIGMA = 0.1;

// per-branch LDS record (doubles)
enum {
  BR_PF = 0, BR_QF, BR_PT, BR_QT,
  BR_HF, BR_HT,                 // flow inequality values (or 0)
  BR_JPF = 6,                   // dPf (4), dQf (4), dPt (4), dQt (4): canonical order
  BR_GL = 22,                   // grad L contribution (4)
  BR_GN = 26,                   // N contribution (4)
  BR_H = 30,                    // Hessian block, packed (10)
  BR_REC = 40
};

__device__ inline bool finite(double v) { return __builtin_isfinite(v); }

struct Views {
  double *x, *lam, *z, *mu;
  const uint8_t *bus_on, *br_on, *gen_on;
  const double *pd, *qd;
  double* K;
};

__device__ inline Views views(const Slots& s, int slot, int nb, int nl, int ng) {
  Views v;
  v.x = s.x + (size_t)slot * s.nx;
  v.lam = s.lam + (size_t)slot * s.neq;
  v.z = s.z + (size_t)slot * s.ni;
  v.mu = s.mu + (size_t)slot * s.ni;
  v.bus_on = s.bus_on + (size_t)slot * nb;
  v.br_on = s.br_on + (size_t)slot * nl;
  v.gen_on = s.gen_on + (size_t)slot * ng;
  v.pd = s.pd + (size_t)slot * nb;
  v.qd = s.qd + (size_t)slot * nb;
  v.K = s.K + (size_t)slot * s.k_stride;
  return v;
}

// powers at both ends of branch l; the to-end arrays are in own order
__device__ inline void branch_powers(const DevNet& net, const double* x, int l,
                                     EndPower& ef, EndPower& et) {
  const int nb = net.nb;
  const int f = net.br_f[l], t = net.br_t[l];
  const double thf = x[f], tht = x[t], vf = x[nb + f], vt = x[nb + t];
  end_power(vf, vt, thf - tht, net.yff_re[l], net.yff_im[l], net.yft_re[l],
            net.yft_im[l], ef);
  end_power(vt, vf, tht - thf, net.ytt_re[l], net.ytt_im[l], net.ytf_re[l],
            net.ytf_im[l], et);
}

__device__ inline double rmax(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < OPF_THREADS / 64; ++w) r = fmax(r, red[w]);
  return r;
}
__device__ inline double rmin(double v, double* red) { return -rmax(-v, red); }
__device__ inline double rsum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < OPF_THREADS / 64; ++w) r += red[w];
  return r;
}
__device__ inline int risum(int v, int* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  int r = 0;
  for (int w = 0; w < OPF_THREADS / 64; ++w) r += red[w];
  return r;
}

// ---------------------------------------------------------------- setup
__global__ __launch_bounds__(OPF_THREADS) void k_setup(DevNet net, Slots s,
                                                       int count, const int* __restrict__ outages,
                                                       int width,
                                                       const double* __restrict__ load_scale,
                                                       const int* __restrict__ item_req) {
  const int slot = blockIdx.x;
  if (slot >= count) return;
  SlotState& S = s.st[slot];
  if (S.phase != PH_NEW) return;
  const int nb = net.nb, nl = net.nl, ng = net.ng;
  const int tid = threadIdx.x;
  __shared__ double red[OPF_THREADS / 64];
  __shared__ int ired[OPF_THREADS / 64];
  const long long scen = S.scen;
  const int o0 = outages[width * scen], o1 = outages[width * scen + 1];
  const int o2 = width > 2 ? outages[width * scen + 2] : -1;
  const int main = S.main_label;
  const int* label = s.label + (size_t)slot * nb;
  Views v = views(s, slot, nb, nl, ng);
  uint8_t* bus_on = const_cast<uint8_t*>(v.bus_on);
  uint8_t* br_on = const_cast<uint8_t*>(v.br_on);
  uint8_t* gen_on = const_cast<uint8_t*>(v.gen_on);
  double* pd = const_cast<double*>(v.pd);
  double* qd = const_cast<double*>(v.qd);
  const int load0 = nl + ng;
  // a served request's own load snapshot: every load scaled by its factor
  const double* scale = (load_scale != nullptr && item_req != nullptr)
                            ? load_scale + (size_t)item_req[scen] * net.nd
                            : nullptr;
  int cnt = 0;
  for (int b = tid; b < nb; b += OPF_THREADS) {
    const bool on = label[b] == main;
    bus_on[b] = on;
    double p = 0.0, q = 0.0;
    if (on) {
      for (int e = net.bus_load_ptr[b]; e < net.bus_load_ptr[b + 1]; ++e) {
        const int d = net.bus_load[e];
        if (load0 + d == o0 || load0 + d == o1 || load0 + d == o2) continue;
        if (scale != nullptr) {
          p += net.pd[d] * scale[d];
          q += net.qd[d] * scale[d];
        } else {
          p += net.pd[d];
          q += net.qd[d];
        }
      }
      cnt += 2;
    }
    pd[b] = p;
    qd[b] = q;
    v.x[b] = 0.0;
    v.x[nb + b] = on ? fmin(fmax(1.0, net.vmin[b]), net.vmax[b]) : 1.0;
  }
  int ngon = 0;
  for (int g = tid; g < ng; g += OPF_THREADS) {
    const bool on = (nl + g != o0) && (nl + g != o1) && (nl + g != o2) &&
                    (label[net.gen_bus[g]] == main);
    gen_on[g] = on;
    ngon += on;
    v.x[2 * nb + g] = on ? 0.5 * (net.pmin[g] + net.pmax[g]) : 0.0;
    v.x[2 * nb + ng + g] = on ? 0.5 * (net.qmin[g] + net.qmax[g]) : 0.0;
    cnt += on ? 4 : 0;
  }
  for (int l = tid; l < nl; l += OPF_THREADS) {
    const bool on = (l != o0) && (l != o1) && (l != o2) && (label[net.br_f[l]] == main);
    br_on[l] = on;
    if (on && net.rate[l] > 0.0) cnt += 2;
  }
  for (int i = tid; i < s.neq; i += OPF_THREADS) v.lam[i] = 0.0;
  const int n_ineq = risum(cnt, ired);
  const int n_gen_on = risum(ngon, ired);
  __syncthreads();
  // initial slacks z = max(-h, 1), mu = gamma / z with gamma = 1
  const int ni = s.ni;
  for (int i = tid; i < ni; i += OPF_THREADS) { v.z[i] = 1.0; v.mu[i] = 0.0; }
  __syncthreads();
  for (int l = tid; l < nl; l += OPF_THREADS) {
    if (!br_on[l] || !(net.rate[l] > 0.0)) continue;
    EndPower ef, et;
    branch_powers(net, v.x, l, ef, et);
    const double r2 = net.rate[l] * net.rate[l];
    const double hf = ef.P * ef.P + ef.Q * ef.Q - r2;
    const double ht = et.P * et.P + et.Q * et.Q - r2;
    v.z[l] = fmax(-hf, 1.0);
    v.z[nl + l] = fmax(-ht, 1.0);
  }
  for (int b = tid; b < nb; b += OPF_THREADS) {
    if (!bus_on[b]) continue;
    const double vm = v.x[nb + b];
    v.z[2 * nl + b] = fmax(-(net.vmin[b] - vm), 1.0);
    v.z[2 * nl + nb + b] = fmax(-(vm - net.vmax[b]), 1.0);
  }
  double cost = 0.0;
  for (int g = tid; g < ng; g += OPF_THREADS) {
    if (!gen_on[g]) continue;
    const double pg = v.x[2 * nb + g], qg = v.x[2 * nb + ng + g];
    const int o = 2 * nl + 2 * nb;
    v.z[o + g] = fmax(-(net.pmin[g] - pg), 1.0);
    v.z[o + ng + g] = fmax(-(pg - net.pmax[g]), 1.0);
    v.z[o + 2 * ng + g] = fmax(-(net.qmin[g] - qg), 1.0);
    v.z[o + 3 * ng + g] = fmax(-(qg - net.qmax[g]), 1.0);
    const double p = net.base_mva * pg;
    cost += net.c2[g] * p * p + net.c1[g] * p + net.c0[g];
  }
  const double f0 = rsum(cost, red);
  __syncthreads();
  // mu = 1 / z on active inequalities
  for (int l = tid; l < nl; l += OPF_THREADS)
    if (br_on[l] && net.rate[l] > 0.0) { v.mu[l] = 1.0 / v.z[l]; v.mu[nl + l] = 1.0 / v.z[nl + l]; }
  for (int b = tid; b < nb; b += OPF_THREADS)
    if (bus_on[b]) {
      v.mu[2 * nl + b] = 1.0 / v.z[2 * nl + b];
      v.mu[2 * nl + nb + b] = 1.0 / v.z[2 * nl + nb + b];
    }
  for (int g = tid; g < ng; g += OPF_THREADS)
    if (gen_on[g])
      for (int k = 0; k < 4; ++k) {
        const int i = 2 * nl + 2 * nb + k * ng + g;
        v.mu[i] = 1.0 / v.z[i];
      }
  __syncthreads();
  if (tid == 0) {
    S.n_ineq = n_ineq;
    S.gamma = 1.0;
    S.f = f0;
    S.f_prev = f0;
    S.iters = 0;
    S.job = 0;
    if (S.ref_bus < 0 || n_gen_on == 0) {
      S.phase = PH_DONE;
      S.status = OPF_NOT_RUN;
      S.cause |= C_OPF;
      S.f = __builtin_nan("");
    } else {
      S.phase = PH_IPM;
      S.status = OPF_MAXIT;
    }
  }
}

// ------------------------------------------------------- evaluate + assemble
__global__ __launch_bounds__(OPF_THREADS) void k_opf_eval(DevNet net, Slots s,
                                                          int count, double tol,
                                                          int max_it, const int* __restrict__ list) {
  const int slot = list_slot(list, count);
  if (slot < 0) return;
  SlotState& S = s.st[slot];
  if (S.phase != PH_IPM) return;
  const int nb = net.nb, nl = net.nl, ng = net.ng;
  const int nx = s.nx, nk = s.nk, ldk = s.ldk;
  const int tid = threadIdx.x;
  extern __shared__ double sh[];
  double* br = sh;                          // [nl][BR_REC]
  double* gv = br + (size_t)nl * BR_REC;    // [2nb] balance residual
  double* gL = gv + 2 * nb;                 // [nx]
  double* gN = gL + nx;                     // [nx]
  __shared__ double red[OPF_THREADS / 64];
  __shared__ int s_job;
  Views v = views(s, slot, nb, nl, ng);
  const int ref = S.ref_bus;
  const double gamma = S.gamma;
  const int iters = S.iters;
  bool bad = false;

  // ---- branch terms
  for (int l = tid; l < nl; l += OPF_THREADS) {
    double* R = br + (size_t)l * BR_REC;
    if (!v.br_on[l]) {
      for (int k = 0; k < BR_REC; ++k) R[k] = 0.0;
      continue;
    }
    const int f = net.br_f[l], t = net.br_t[l];
    EndPower e[2];
    branch_powers(net, v.x, l, e[0], e[1]);
    const double vf = v.x[nb + f], vt = v.x[nb + t];
    const bool rated = net.rate[l] > 0.0;
    const double r2 = net.rate[l] * net.rate[l];
    double Hc[10], gLc[4], gNc[4];
    for (int k = 0; k < 10; ++k) Hc[k] = 0.0;
    for (int k = 0; k < 4; ++k) { gLc[k] = 0.0; gNc[k] = 0.0; }
    for (int side = 0; side < 2; ++side) {
      const EndPower& E = e[side];
      const int own = side ? t : f;
      const double vo = side ? vt : vf, vr = side ? vf : vt;
      const double goo = side ? net.ytt_re[l] : net.yff_re[l];
      const double boo = side ? net.ytt_im[l] : net.yff_im[l];
      double HP[10], HQ[10], Hown[10], dh[4], gl[4], gn[4];
      end_hessians(vo, vr, goo, boo, E, HP, HQ);
      const double lp = v.lam[own], lq = v.lam[nb + own];
      for (int k = 0; k < 10; ++k) Hown[k] = lp * HP[k] + lq * HQ[k];
      for (int k = 0; k < 4; ++k) { gl[k] = lp * E.dP[k] + lq * E.dQ[k]; gn[k] = gl[k]; }
      double h = 0.0;
      if (rated) {
        h = E.P * E.P + E.Q * E.Q - r2;
        const int ii = side ? nl + l : l;
        const double mu = v.mu[ii], z = v.z[ii];
        const double wn = mu + (gamma + mu * h) / z;
        const double d = mu / z;
        for (int k = 0; k < 4; ++k) dh[k] = 2.0 * (E.P * E.dP[k] + E.Q * E.dQ[k]);
        for (int i = 0; i < 4; ++i)
          for (int j = i; j < 4; ++j) {
            const int p = pk(i, j);
            const double outer = E.dP[i] * E.dP[j] + E.dQ[i] * E.dQ[j];
            Hown[p] += mu * 2.0 * (outer + E.P * HP[p] + E.Q * HQ[p]) + d * dh[i] * dh[j];
          }
        for (int k = 0; k < 4; ++k) { gl[k] += mu * dh[k]; gn[k] += wn * dh[k]; }
      }
      R[side ? BR_HT : BR_HF] = h;
      if (rated) {
        // the step update reuses exactly these values (see k_opf_update)
        double* hv = s.hv + (size_t)slot * s.ni;
        double* jh = s.jh + ((size_t)slot * nl + l) * 8 + 4 * side;
        hv[side ? nl + l : l] = h;
        const int pm[4] = {side ? 1 : 0, side ? 0 : 1, side ? 3 : 2, side ? 2 : 3};
        for (int k = 0; k < 4; ++k) jh[pm[k]] = dh[k];
      }
      // own order -> canonical (theta_f, theta_t, V_f, V_t)
      const int perm[4] = {side ? 1 : 0, side ? 0 : 1, side ? 3 : 2, side ? 2 : 3};
      for (int i = 0; i < 4; ++i) {
        gLc[perm[i]] += gl[i];
        gNc[perm[i]] += gn[i];
        R[BR_JPF + 8 * side + perm[i]] = E.dP[i];
        R[BR_JPF + 8 * side + 4 + perm[i]] = E.dQ[i];
        for (int j = i; j < 4; ++j) Hc[pk(perm[i], perm[j])] += Hown[pk(i, j)];
      }
    }
    R[BR_PF] = e[0].P; R[BR_QF] = e[0].Q; R[BR_PT] = e[1].P; R[BR_QT] = e[1].Q;
    for (int k = 0; k < 4; ++k) { R[BR_GL + k] = gLc[k]; R[BR_GN + k] = gNc[k]; }
    for (int k = 0; k < 10; ++k) R[BR_H + k] = Hc[k];
  }
  __syncthreads();

  // ---- bus rows: balance residual, gradient entries
  const int bo = 2 * nl;                    // first V-box inequality
  for (int b = tid; b < nb; b += OPF_THREADS) {
    if (!v.bus_on[b]) { gv[b] = gv[nb + b] = 0.0; gL[b] = gL[nb + b] = gN[b] = gN[nb + b] = 0.0; continue; }
    const double vm = v.x[nb + b];
    double P = net.gs[b] * vm * vm, Q = -net.bs[b] * vm * vm;
    double lt = 0.0, lv = 0.0, nt = 0.0, nv = 0.0;
    for (int e = net.bus_br_ptr[b]; e < net.bus_br_ptr[b + 1]; ++e) {
      const int l = net.bus_br[e];
      if (!v.br_on[l]) continue;
      const double* R = br + (size_t)l * BR_REC;
      const bool isf = net.br_f[l] == b;
      P += isf ? R[BR_PF] : R[BR_PT];
      Q += isf ? R[BR_QF] : R[BR_QT];
      const int it = isf ? 0 : 1, iv = isf ? 2 : 3;
      lt += R[BR_GL + it]; lv += R[BR_GL + iv];
      nt += R[BR_GN + it]; nv += R[BR_GN + iv];
    }
    double pg = 0.0, qg = 0.0;
    for (int e = net.bus_gen_ptr[b]; e < net.bus_gen_ptr[b + 1]; ++e) {
      const int g = net.bus_gen[e];
      if (!v.gen_on[g]) continue;
      pg += v.x[2 * nb + g];
      qg += v.x[2 * nb + ng + g];
    }
    gv[b] = P + v.pd[b] - pg;
    gv[nb + b] = Q + v.qd[b] - qg;
    const double lp = v.lam[b], lq = v.lam[nb + b];
    const double sh_v = lp * 2.0 * net.gs[b] * vm - lq * 2.0 * net.bs[b] * vm;
    const double mlo = v.mu[bo + b], mhi = v.mu[bo + nb + b];
    const double zlo = v.z[bo + b], zhi = v.z[bo + nb + b];
    const double hlo = net.vmin[b] - vm, hhi = vm - net.vmax[b];
    s.hv[(size_t)slot * s.ni + bo + b] = hlo;
    s.hv[(size_t)slot * s.ni + bo + nb + b] = hhi;
    const double wlo = mlo + (gamma + mlo * hlo) / zlo, whi = mhi + (gamma + mhi * hhi) / zhi;
    gL[b] = (b == ref) ? 0.0 : lt;
    gN[b] = (b == ref) ? 0.0 : nt;
    gL[nb + b] = lv + sh_v + (mhi - mlo);
    gN[nb + b] = nv + sh_v + (whi - wlo);
  }
  const int go = 2 * nl + 2 * nb;           // first Pmin inequality
  for (int g = tid; g < ng; g += OPF_THREADS) {
    const int ip = 2 * nb + g, iq = 2 * nb + ng + g;
    if (!v.gen_on[g]) { gL[ip] = gL[iq] = gN[ip] = gN[iq] = 0.0; continue; }
    const int k = net.gen_bus[g];
    const double pg = v.x[ip], qg = v.x[iq];
    const double df = 2.0 * net.c2[g] * net.base_mva * net.base_mva * pg + net.c1[g] * net.base_mva;
    double m[4], w[4];
    const double h[4] = {net.pmin[g] - pg, pg - net.pmax[g], net.qmin[g] - qg, qg - net.qmax[g]};
    for (int j = 0; j < 4; ++j) {
      s.hv[(size_t)slot * s.ni + go + j * ng + g] = h[j];
      m[j] = v.mu[go + j * ng + g];
      w[j] = m[j] + (gamma + m[j] * h[j]) / v.z[go + j * ng + g];
    }
    gL[ip] = df - v.lam[k] + (m[1] - m[0]);
    gN[ip] = df - v.lam[k] + (w[1] - w[0]);
    gL[iq] = -v.lam[nb + k] + (m[3] - m[2]);
    gN[iq] = -v.lam[nb + k] + (w[3] - w[2]);
  }
  __syncthreads();

  // ---- termination measures
  double mg = 0.0, mh = -__builtin_inf(), mx = 0.0, mz = 0.0, ml = 0.0, mm = 0.0, mgl = 0.0;
  double zmu = 0.0, cost = 0.0, viol = -__builtin_inf();
  for (int b = tid; b < nb; b += OPF_THREADS) {
    if (!v.bus_on[b]) continue;
    mg = fmax(mg, fmax(fabs(gv[b]), fabs(gv[nb + b])));
    mx = fmax(mx, fmax(fabs(v.x[b]), fabs(v.x[nb + b])));
    ml = fmax(ml, fmax(fabs(v.lam[b]), fabs(v.lam[nb + b])));
    mgl = fmax(mgl, fmax(fabs(gL[b]), fabs(gL[nb + b])));
    bad |= !finite(gv[b]) || !finite(gv[nb + b]) || !finite(gN[b]) || !finite(gN[nb + b]);
    const double vm = v.x[nb + b];
    for (int j = 0; j < 2; ++j) {
      const int i = bo + j * nb + b;
      const double h = j ? vm - net.vmax[b] : net.vmin[b] - vm;
      mh = fmax(mh, h);
      mz = fmax(mz, fabs(v.z[i]));
      mm = fmax(mm, fabs(v.mu[i]));
      zmu += v.z[i] * v.mu[i];
    }
    viol = fmax(viol, fmax(vm - net.vmax[b], net.vmin[b] - vm));
  }
  for (int g = tid; g < ng; g += OPF_THREADS) {
    if (!v.gen_on[g]) continue;
    const double pg = v.x[2 * nb + g], qg = v.x[2 * nb + ng + g];
    mx = fmax(mx, fmax(fabs(pg), fabs(qg)));
    mgl = fmax(mgl, fmax(fabs(gL[2 * nb + g]), fabs(gL[2 * nb + ng + g])));
    bad |= !finite(gN[2 * nb + g]) || !finite(gN[2 * nb + ng + g]);
    const double h[4] = {net.pmin[g] - pg, pg - net.pmax[g], net.qmin[g] - qg, qg - net.qmax[g]};
    for (int j = 0; j < 4; ++j) {
      const int i = go + j * ng + g;
      mh = fmax(mh, h[j]);
      mz = fmax(mz, fabs(v.z[i]));
      mm = fmax(mm, fabs(v.mu[i]));
      zmu += v.z[i] * v.mu[i];
      viol = fmax(viol, h[j]);
    }
    const double p = net.base_mva * pg;
    cost += net.c2[g] * p * p + net.c1[g] * p + net.c0[g];
  }
  for (int l = tid; l < nl; l += OPF_THREADS) {
    if (!v.br_on[l] || !(net.rate[l] > 0.0)) continue;
    const double* R = br + (size_t)l * BR_REC;
    for (int j = 0; j < 2; ++j) {
      const int i = j ? nl + l : l;
      mh = fmax(mh, R[j ? BR_HT : BR_HF]);
      mz = fmax(mz, fabs(v.z[i]));
      mm = fmax(mm, fabs(v.mu[i]));
      zmu += v.z[i] * v.mu[i];
    }
    const double sf = sqrt(R[BR_PF] * R[BR_PF] + R[BR_QF] * R[BR_QF]);
    const double st = sqrt(R[BR_PT] * R[BR_PT] + R[BR_QT] * R[BR_QT]);
    viol = fmax(viol, fmax(sf, st) - net.rate[l]);
  }
  mg = rmax(mg, red); mh = rmax(mh, red); mx = rmax(mx, red); mz = rmax(mz, red);
  ml = rmax(ml, red); mm = rmax(mm, red); mgl = rmax(mgl, red); viol = rmax(viol, red);
  zmu = rsum(zmu, red);
  cost = rsum(cost, red);
  const double nbad = rmax(bad ? 1.0 : 0.0, red);
  if (tid == 0) {
    const double fprev = S.f_prev;
    const double feas = fmax(mg, mh) / (1.0 + fmax(mx, mz));
    const double grad = mgl / (1.0 + fmax(ml, mm));
    const double comp = zmu / (1.0 + mx);
    const double dcost = fabs(cost - fprev) / (1.0 + fabs(fprev));
    S.metrics[0] = feas; S.metrics[1] = grad; S.metrics[2] = comp; S.metrics[3] = dcost;
    S.f = cost;
    const double mmax = fmax(fmax(feas, grad), fmax(comp, dcost));
    const bool fin = finite(feas) && finite(grad) && finite(comp) && finite(dcost);
    int job = 0;
    if (iters > 0 && fin && mmax < tol) {
      S.status = OPF_CONVERGED;
      S.phase = PH_DYN;
      S.max_viol = viol;
    } else if (iters >= max_it) {
      S.status = OPF_MAXIT;
      S.phase = PH_DONE;
    } else if (nbad > 0.0 || !fin) {
      S.status = OPF_NUMERICAL;      // the step that could not be assembled counts
      S.phase = PH_DONE;
      S.iters = iters + 1;
    } else {
      job = 1;
    }
    S.job = job;
    s_job = job;
  }
  __syncthreads();
  if (!s_job) return;

  // ---- assemble the KKT system (column-major, rhs in column nk)
  double* K = v.K;
  {
    const size_t total = (size_t)nk * ldk;
    double2* K2 = reinterpret_cast<double2*>(K);
    const double2 zero2 = {0.0, 0.0};
    for (size_t i = tid; i < total / 2; i += OPF_THREADS) K2[i] = zero2;
    if ((total & 1) && tid == 0) K[total - 1] = 0.0;
  }
  __syncthreads();
#define KK(r, c) K[(size_t)(r) * ldk + (c)]
#define RHS(r) K[(size_t)(r) * ldk + nk]
  bool badw = false;
  for (int b = tid; b < nb; b += OPF_THREADS) {
    const int rt = b, rv = nb + b, rp = nx + b, rq = nx + nb + b;
    if (!v.bus_on[b]) {
      KK(rt, rt) = 1.0; KK(rv, rv) = 1.0; KK(rp, rp) = 1.0; KK(rq, rq) = 1.0;
      continue;
    }
    const bool isref = (b == ref);
    const double vm = v.x[nb + b];
    double Htt = 0.0, Htv = 0.0, Hvv = 0.0;
    double Jpt = 0.0, Jpv = 2.0 * net.gs[b] * vm, Jqt = 0.0, Jqv = -2.0 * net.bs[b] * vm;
    for (int e = net.bus_br_ptr[b]; e < net.bus_br_ptr[b + 1]; ++e) {
      const int l = net.bus_br[e];
      if (!v.br_on[l]) continue;
      const double* R = br + (size_t)l * BR_REC;
      const bool isf = net.br_f[l] == b;
      const int r = isf ? net.br_t[l] : net.br_f[l];
      const int ot = isf ? 0 : 1, ov = isf ? 2 : 3;    // own indices
      const int xt = isf ? 1 : 0, xv = isf ? 3 : 2;    // other indices
      const double* H = R + BR_H;
      const double* dP = R + BR_JPF + (isf ? 0 : 8);
      const double* dQ = dP + 4;
      Htt += H[pk(ot, ot)]; Htv += H[pk(ot, ov)]; Hvv += H[pk(ov, ov)];
      Jpt += dP[ot]; Jpv += dP[ov]; Jqt += dQ[ot]; Jqv += dQ[ov];
      const bool rref = (r == ref);
      // M rows theta_b, V_b; columns of the other bus
      if (!isref) {
        if (!rref) KK(rt, r) += H[pk(ot, xt)];
        KK(rt, nb + r) += H[pk(ot, xv)];
      }
      if (!rref) KK(rv, r) += H[pk(ov, xt)];
      KK(rv, nb + r) += H[pk(ov, xv)];
      // Jg rows P_b, Q_b and the transposed columns
      if (!rref) {
        KK(rp, r) += dP[xt]; KK(r, rp) += dP[xt];
        KK(rq, r) += dQ[xt]; KK(r, rq) += dQ[xt];
      }
      KK(rp, nb + r) += dP[xv]; KK(nb + r, rp) += dP[xv];
      KK(rq, nb + r) += dQ[xv]; KK(nb + r, rq) += dQ[xv];
    }
    Hvv += v.lam[b] * 2.0 * net.gs[b] - v.lam[nb + b] * 2.0 * net.bs[b];
    Hvv += v.mu[bo + b] / v.z[bo + b] + v.mu[bo + nb + b] / v.z[bo + nb + b];
    if (isref) {
      KK(rt, rt) = 1.0;
    } else {
      KK(rt, rt) = Htt; KK(rt, rv) = Htv; KK(rv, rt) = Htv;
      KK(rp, rt) = Jpt; KK(rt, rp) = Jpt; KK(rq, rt) = Jqt; KK(rt, rq) = Jqt;
    }
    KK(rv, rv) = Hvv;
    KK(rp, rv) = Jpv; KK(rv, rp) = Jpv; KK(rq, rv) = Jqv; KK(rv, rq) = Jqv;
    RHS(rt) = isref ? 0.0 : -gN[b];
    RHS(rv) = -gN[nb + b];
    RHS(rp) = -gv[b];
    RHS(rq) = -gv[nb + b];
    badw |= !finite(Htt) || !finite(Htv) || !finite(Hvv);
  }
  for (int g = tid; g < ng; g += OPF_THREADS) {
    const int ip = 2 * nb + g, iq = 2 * nb + ng + g;
    if (!v.gen_on[g]) { KK(ip, ip) = 1.0; KK(iq, iq) = 1.0; continue; }
    const int k = net.gen_bus[g];
    double dpp = 2.0 * net.c2[g] * net.base_mva * net.base_mva;
    dpp += v.mu[go + g] / v.z[go + g] + v.mu[go + ng + g] / v.z[go + ng + g];
    const double dqq = v.mu[go + 2 * ng + g] / v.z[go + 2 * ng + g] +
                       v.mu[go + 3 * ng + g] / v.z[go + 3 * ng + g];
    KK(ip, ip) = dpp;
    KK(iq, iq) = dqq;
    KK(nx + k, ip) = -1.0; KK(ip, nx + k) = -1.0;
    KK(nx + nb + k, iq) = -1.0; KK(iq, nx + nb + k) = -1.0;
    RHS(ip) = -gN[ip];
    RHS(iq) = -gN[iq];
    badw |= !finite(dpp) || !finite(dqq);
  }
  for (int l = tid; l < nl; l += OPF_THREADS) {
    const double* R = br + (size_t)l * BR_REC;
    for (int k = 0; k < 10; ++k) badw |= !finite(R[BR_H + k]);
  }
#undef KK
#undef RHS
  const double nbw = rmax(badw ? 1.0 : 0.0, red);
  if (tid == 0 && nbw > 0.0) {
    S.status = OPF_NUMERICAL;
    S.phase = PH_DONE;
    S.job = 0;
    S.iters = iters + 1;
  }
}

// ------------------------------------------------------------------ update
__global__ __launch_bounds__(OPF_THREADS) void k_opf_update(DevNet net, Slots s,
                                                            int count,
                                                            double gamma_max,
                                                            const int* __restrict__ list) {
  const int slot = list_slot(list, count);
  if (slot < 0) return;
  SlotState& S = s.st[slot];
  if (S.phase != PH_IPM || S.job == 0) return;
  const int nb = net.nb, nl = net.nl, ng = net.ng;
  const int nx = s.nx, nk = s.nk, ldk = s.ldk, ni = s.ni;
  const int tid = threadIdx.x;
  __shared__ double red[OPF_THREADS / 64];
  extern __shared__ double dz[];            // [ni], then the solution [nk]
  double* d = dz + ni;
  Views v = views(s, slot, nb, nl, ng);
  for (int i = tid; i < nk; i += OPF_THREADS) d[i] = v.K[(size_t)i * ldk + nk];
  const double gamma = S.gamma;
  const int ref = S.ref_bus;
  bool bad = S.singular != 0;
  for (int i = tid; i < nk; i += OPF_THREADS) bad |= !finite(d[i]);
  // dz = -h - z - Jh dx on active inequalities (0 elsewhere)
  for (int i = tid; i < ni; i += OPF_THREADS) dz[i] = 0.0;
  __syncthreads();
  // The values of h and grad h are the ones the evaluation used to build
  // the right-hand side, so the rounding in h cancels between N and dz the
  // way it does in exact arithmetic (recomputing h here could round
  // differently, and near the optimum that difference is amplified by mu/z).
  const double* hv = s.hv + (size_t)slot * ni;
  for (int l = tid; l < nl; l += OPF_THREADS) {
    if (!v.br_on[l] || !(net.rate[l] > 0.0)) continue;
    const int f = net.br_f[l], t = net.br_t[l];
    const double* jh = s.jh + ((size_t)slot * nl + l) * 8;
    const double dc[4] = {d[f], d[t], d[nb + f], d[nb + t]};
    for (int side = 0; side < 2; ++side) {
      double jd = 0.0;
      for (int k = 0; k < 4; ++k) jd += jh[4 * side + k] * dc[k];
      const int i = side ? nl + l : l;
      dz[i] = -hv[i] - v.z[i] - jd;
    }
  }
  const int bo = 2 * nl, go = 2 * nl + 2 * nb;
  for (int b = tid; b < nb; b += OPF_THREADS) {
    if (!v.bus_on[b]) continue;
    const double dv = d[nb + b];
    dz[bo + b] = -hv[bo + b] - v.z[bo + b] + dv;
    dz[bo + nb + b] = -hv[bo + nb + b] - v.z[bo + nb + b] - dv;
  }
  for (int g = tid; g < ng; g += OPF_THREADS) {
    if (!v.gen_on[g]) continue;
    const double dp = d[2 * nb + g], dq = d[2 * nb + ng + g];
    dz[go + g] = -hv[go + g] - v.z[go + g] + dp;
    dz[go + ng + g] = -hv[go + ng + g] - v.z[go + ng + g] - dp;
    dz[go + 2 * ng + g] = -hv[go + 2 * ng + g] - v.z[go + 2 * ng + g] + dq;
    dz[go + 3 * ng + g] = -hv[go + 3 * ng + g] - v.z[go + 3 * ng + g] - dq;
  }
  __syncthreads();
  // step lengths; an inequality is active iff mu > 0 or it was set up (z, mu
  // of masked entries are 1, 0 and dz = 0, so they never bind)
  double ap = __builtin_inf(), ad = __builtin_inf();
  for (int i = tid; i < ni; i += OPF_THREADS) {
    const double z = v.z[i], mu = v.mu[i];
    if (mu == 0.0 && dz[i] == 0.0) continue;
    const double dmu = -mu + (gamma - mu * dz[i]) / z;
    if (dz[i] < 0.0) ap = fmin(ap, -z / dz[i]);
    if (dmu < 0.0) ad = fmin(ad, -mu / dmu);
    bad |= !finite(dz[i]) || !finite(dmu);
  }
  ap = rmin(ap, red);
  ad = rmin(ad, red);
  const double nbad = rmax(bad ? 1.0 : 0.0, red);
  if (nbad > 0.0) {
    if (tid == 0) { S.status = OPF_NUMERICAL; S.phase = PH_DONE; S.job = 0; S.iters += 1; }
    return;
  }
  const double alpha_p = fmin(XI * ap, 1.0);
  const double alpha_d = fmin(XI * ad, 1.0);
  __syncthreads();
  // update
  double zmu = 0.0;
  bool bad2 = false;
  for (int i = tid; i < ni; i += OPF_THREADS) {
    const double z = v.z[i], mu = v.mu[i];
    if (mu == 0.0 && dz[i] == 0.0) continue;
    const double dmu = -mu + (gamma - mu * dz[i]) / z;
    const double zn = z + alpha_p * dz[i];
    const double mn = mu + alpha_d * dmu;
    v.z[i] = zn;
    v.mu[i] = mn;
    zmu += zn * mn;
    bad2 |= !finite(zn) || !finite(mn);
  }
  for (int b = tid; b < nb; b += OPF_THREADS) {
    if (!v.bus_on[b]) continue;
    if (b != ref) v.x[b] += alpha_p * d[b];
    v.x[nb + b] += alpha_p * d[nb + b];
    v.lam[b] += alpha_d * d[nx + b];
    v.lam[nb + b] += alpha_d * d[nx + nb + b];
    bad2 |= !finite(v.x[b]) || !finite(v.x[nb + b]) || !finite(v.lam[b]) || !finite(v.lam[nb + b]);
  }
  for (int g = tid; g < ng; g += OPF_THREADS) {
    if (!v.gen_on[g]) continue;
    v.x[2 * nb + g] += alpha_p * d[2 * nb + g];
    v.x[2 * nb + ng + g] += alpha_p * d[2 * nb + ng + g];
    bad2 |= !finite(v.x[2 * nb + g]) || !finite(v.x[2 * nb + ng + g]);
  }
  zmu = rsum(zmu, red);
  const double nbad2 = rmax(bad2 ? 1.0 : 0.0, red);
  if (tid == 0) {
    S.iters += 1;
    S.job = 0;
    S.f_prev = S.f;
    const double gnew = (S.n_ineq > 0) ? SIGMA * zmu / S.n_ineq : gamma;
    S.gamma = gnew;
    if (!(gnew <= gamma_max) || nbad2 > 0.0) {
      S.status = OPF_NUMERICAL;
      S.phase = PH_DONE;
    }
  }
}

size_t opf_eval_lds(int nb, int nl, int ng) {
  const int nx = 2 * nb + 2 * ng;
  return sizeof(double) * ((size_t)nl * BR_REC + 2 * nb + 2 * nx);
}

void opf_set_attrs(size_t bytes) {
  hipFuncSetAttribute(reinterpret_cast<const void*>(k_opf_eval),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  hipFuncSetAttribute(reinterpret_cast<const void*>(k_opf_update),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

void launch_setup_k(const DevNet& net, const Slots& s, int count,
                    const int* outages, hipStream_t st, int width, const double* load_scale,
                    const int* item_req) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_setup, dim3(count), dim3(OPF_THREADS), 0, st, net, s,
                     count, outages, width, load_scale, item_req);
}

void launch_opf_eval(const DevNet& net, const Slots& s, int count, double tol,
                     int max_it, hipStream_t st, const JobList& jl) {
  const int grid = job_grid(count, jl);
  if (grid <= 0) return;
  hipLaunchKernelGGL(k_opf_eval, dim3(grid), dim3(OPF_THREADS),
                     opf_eval_lds(net.nb, net.nl, net.ng), st, net, s, count,
                     tol, max_it, jl.list);
}

void launch_opf_update(const DevNet& net, const Slots& s, int count,
                       double gamma_max, hipStream_t st, const JobList& jl) {
  const int grid = job_grid(count, jl);
  if (grid <= 0) return;
  hipLaunchKernelGGL(k_opf_update, dim3(grid), dim3(OPF_THREADS),
                     sizeof(double) * (size_t)(s.ni + s.nk), st, net, s, count, gamma_max,
                     jl.list);
}

}  // namespace cs
