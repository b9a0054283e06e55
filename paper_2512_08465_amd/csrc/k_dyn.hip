// Linearised state matrix at the OPF point (Section II.B.2).
//
// Device models: two-axis synchronous machine (delta, omega, Eq', Ed') with a
// first-order AVR (Efd) and a governor-turbine (Psv, Pm), stator algebraic
// equations, constant-impedance loads at the OPF voltage, and the network
// balance; A = f_x - f_y g_y^{-1} g_x.
//
// k_dyn_assemble writes, per scenario, the algebraic Jacobian g_y over
// y = [Id, Iq, theta, V] and the nonzero columns of g_x (delta_j, Eq'_j,
// Ed'_j for every generator j) as right-hand sides; the batched LU kernel
// then leaves X = g_y^{-1} g_x in those columns.  k_form_state builds A for
// the in-service machines of the island: f_x is block diagonal and f_y picks
// at most two rows of X per state, so A_full = f_x - f_y X is a gather.  The
// absolute angles are made relative to the first machine (its delta row is
// subtracted from the others, then its delta row and column are dropped),
// which removes the zero eigenvalue of a uniform angle shift.
//
// Equilibrium from the operating point (V, theta, Pg, Qg) of each machine:
//   I = conj(S / V), E = V + (Rs + j Xq) I, delta = arg E,
//   Id + j Iq = I e^{-j(delta - pi/2)}, Vd + j Vq = V e^{-j(delta - pi/2)},
//   Ed' = Vd + Rs Id - Xq' Iq, Eq' = Vq + Rs Iq + Xd' Id.
#include "cs_internal.h"
#include "branch_math.h"

namespace cs {

constexpr int DYN_THREADS = 256;

struct Machine {
  double delta, Id, Iq, Edp, Eqp, vk, sa, ca;  // sa, ca = sin/cos(delta - theta_k)
};

__device__ inline Machine equilibrium(const DevNet& net, const double* x, int g) {
  const int nb = net.nb, ng = net.ng;
  const int k = net.gen_bus[g];
  const double* p = net.dyn + (size_t)g * kDyn;
  const double Xq = p[3], Xdp = p[4], Xqp = p[5], Rs = p[8];
  const double th = x[k], vm = x[nb + k];
  const double pg = x[2 * nb + g], qg = x[2 * nb + ng + g];
  double sth, cth;
  sincos(th, &sth, &cth);
  const double Vr = vm * cth, Vi = vm * sth;
  // I = conj(S / V) = (P - jQ) / conj(V) = (P - jQ) V / |V|^2
  const double inv = 1.0 / (vm * vm);
  const double Ir = (pg * Vr + qg * Vi) * inv;
  const double Ii = (pg * Vi - qg * Vr) * inv;
  const double Er = Vr + Rs * Ir - Xq * Ii;
  const double Ei = Vi + Rs * Ii + Xq * Ir;
  const double delta = atan2(Ei, Er);
  double sd, cd;
  sincos(delta, &sd, &cd);
  // e^{-j(delta - pi/2)} = sin(delta) + j cos(delta)
  const double Id = Ir * sd - Ii * cd, Iq = Ir * cd + Ii * sd;
  const double Vd = Vr * sd - Vi * cd, Vq = Vr * cd + Vi * sd;
  Machine m;
  m.delta = delta;
  m.Id = Id;
  m.Iq = Iq;
  m.Edp = Vd + Rs * Id - Xqp * Iq;
  m.Eqp = Vq + Rs * Iq + Xdp * Id;
  m.vk = vm;
  sincos(delta - th, &m.sa, &m.ca);
  return m;
}

__global__ __launch_bounds__(DYN_THREADS) void k_dyn_assemble(DevNet net, Slots s, int count) {
  const int slot = blockIdx.x;
  if (slot >= count) return;
  SlotState& S = s.st[slot];
  if (S.phase != PH_DYNB) return;
  const int nb = net.nb, nl = net.nl, ng = net.ng;
  const int ny = s.ny, ldy = s.ldy, nyc = s.nyc;
  const int tid = threadIdx.x;
  const double* x = s.x + (size_t)slot * s.nx;
  const uint8_t* bus_on = s.bus_on + (size_t)slot * nb;
  const uint8_t* br_on = s.br_on + (size_t)slot * nl;
  const uint8_t* gen_on = s.gen_on + (size_t)slot * ng;
  const double* pd = s.pd + (size_t)slot * nb;
  const double* qd = s.qd + (size_t)slot * nb;
  double* K = s.K + (size_t)slot * s.k_stride;
  {
    const size_t total = (size_t)ny * ldy;
    for (size_t i = tid; i < total; i += DYN_THREADS) K[i] = 0.0;
  }
  __syncthreads();
#define YY(r, c) K[(size_t)(r) * ldy + (c)]
  const int cth0 = 2 * ng, cv0 = 2 * ng + nb;
  // stator rows
  for (int g = tid; g < ng; g += DYN_THREADS) {
    if (!gen_on[g]) { YY(g, g) = 1.0; YY(ng + g, ng + g) = 1.0; continue; }
    const Machine m = equilibrium(net, x, g);
    const double* p = net.dyn + (size_t)g * kDyn;
    const double Xdp = p[4], Xqp = p[5], Rs = p[8];
    const int k = net.gen_bus[g];
    YY(g, g) = -Rs;
    YY(g, ng + g) = Xqp;
    YY(g, cth0 + k) = m.vk * m.ca;
    YY(g, cv0 + k) = -m.sa;
    YY(ng + g, g) = -Xdp;
    YY(ng + g, ng + g) = -Rs;
    YY(ng + g, cth0 + k) = -m.vk * m.sa;
    YY(ng + g, cv0 + k) = -m.ca;
    const int c = ny + 3 * g;
    YY(g, c + 0) = -m.vk * m.ca;      // d/d delta
    YY(g, c + 2) = 1.0;               // d/d Ed'
    YY(ng + g, c + 0) = m.vk * m.sa;
    YY(ng + g, c + 1) = 1.0;          // d/d Eq'
  }
  // network rows
  for (int b = tid; b < nb; b += DYN_THREADS) {
    const int rp = cth0 + b, rq = cv0 + b;
    if (!bus_on[b]) { YY(rp, rp) = 1.0; YY(rq, rq) = 1.0; continue; }
    const double vm = x[nb + b];
    double pt = 0.0, pv = 0.0, qt = 0.0, qv = 0.0;
    for (int e = net.bus_gen_ptr[b]; e < net.bus_gen_ptr[b + 1]; ++e) {
      const int g = net.bus_gen[e];
      if (!gen_on[g]) continue;
      const Machine m = equilibrium(net, x, g);
      const double dPdd = m.Id * m.vk * m.ca - m.Iq * m.vk * m.sa;
      const double dQdd = -m.Id * m.vk * m.sa - m.Iq * m.vk * m.ca;
      YY(rp, g) = m.vk * m.sa;
      YY(rp, ng + g) = m.vk * m.ca;
      YY(rq, g) = m.vk * m.ca;
      YY(rq, ng + g) = -m.vk * m.sa;
      pt -= dPdd;
      qt -= dQdd;
      pv += m.Id * m.sa + m.Iq * m.ca;
      qv += m.Id * m.ca - m.Iq * m.sa;
      YY(rp, ny + 3 * g) = dPdd;
      YY(rq, ny + 3 * g) = dQdd;
    }
    // loads: -P0 (V/V0)^2 with V0 = V at the operating point
    pv -= 2.0 * pd[b] / vm;
    qv -= 2.0 * qd[b] / vm;
    // network: minus the derivatives of the bus injection
    pv -= 2.0 * net.gs[b] * vm;
    qv += 2.0 * net.bs[b] * vm;
    for (int e = net.bus_br_ptr[b]; e < net.bus_br_ptr[b + 1]; ++e) {
      const int l = net.bus_br[e];
      if (!br_on[l]) continue;
      const bool isf = net.br_f[l] == b;
      const int r = isf ? net.br_t[l] : net.br_f[l];
      EndPower E;
      if (isf)
        end_power(vm, x[nb + r], x[b] - x[r], net.yff_re[l], net.yff_im[l],
                  net.yft_re[l], net.yft_im[l], E);
      else
        end_power(vm, x[nb + r], x[b] - x[r], net.ytt_re[l], net.ytt_im[l],
                  net.ytf_re[l], net.ytf_im[l], E);
      pt -= E.dP[0]; pv -= E.dP[2]; qt -= E.dQ[0]; qv -= E.dQ[2];
      YY(rp, cth0 + r) -= E.dP[1];
      YY(rp, cv0 + r) -= E.dP[3];
      YY(rq, cth0 + r) -= E.dQ[1];
      YY(rq, cv0 + r) -= E.dQ[3];
    }
    YY(rp, cth0 + b) += pt;
    YY(rp, cv0 + b) += pv;
    YY(rq, cth0 + b) += qt;
    YY(rq, cv0 + b) += qv;
  }
#undef YY
  if (tid == 0) S.job = 1;
}

__global__ __launch_bounds__(DYN_THREADS) void k_form_state(DevNet net, Slots s, int count) {
  const int slot = blockIdx.x;
  if (slot >= count) return;
  SlotState& S = s.st[slot];
  if (S.phase != PH_DYNB) return;
  const int nb = net.nb, ng = net.ng;
  const int ny = s.ny, ldy = s.ldy, lda = s.lda_a;
  const int tid = threadIdx.x;
  extern __shared__ double shd[];
  // per compact machine: fx entries and f_y coefficients
  enum { M_D1, M_Iq, M_Id, M_H2, M_Td, M_Tq, M_TA, M_RTg, M_Tg, M_Tt,
         M_fwId, M_fwIq, M_fqId, M_fdIq, M_feV, M_REC };
  double* mrec = shd;                                  // [ng][M_REC]
  int* gl = reinterpret_cast<int*>(mrec + (size_t)ng * M_REC);   // compact -> gen
  __shared__ int s_nact;
  __shared__ int s_bad;
  const double* x = s.x + (size_t)slot * s.nx;
  const uint8_t* gen_on = s.gen_on + (size_t)slot * ng;
  const double* K = s.K + (size_t)slot * s.k_stride;
  double* A = s.A + (size_t)slot * s.a_stride;
  if (tid == 0) {
    int c = 0;
    for (int g = 0; g < ng; ++g)
      if (gen_on[g]) gl[c++] = g;
    s_nact = c;
    s_bad = S.singular;
  }
  __syncthreads();
  const int nact = s_nact;
  for (int ci = tid; ci < nact; ci += DYN_THREADS) {
    const int g = gl[ci];
    const Machine m = equilibrium(net, x, g);
    const double* p = net.dyn + (size_t)g * kDyn;
    const double H = p[0], D = p[1], Xd = p[2], Xq = p[3], Xdp = p[4], Xqp = p[5];
    const double Td0p = p[6], Tq0p = p[7], KA = p[9], TA = p[10], R = p[11];
    const double Tg = p[12], Tt = p[13];
    const double H2 = 2.0 * H;
    double* r = mrec + (size_t)ci * M_REC;
    r[M_D1] = -D / H2;
    r[M_Iq] = -m.Iq / H2;
    r[M_Id] = -m.Id / H2;
    r[M_H2] = 1.0 / H2;
    r[M_Td] = 1.0 / Td0p;
    r[M_Tq] = 1.0 / Tq0p;
    r[M_TA] = 1.0 / TA;
    r[M_RTg] = -1.0 / (R * Tg);
    r[M_Tg] = 1.0 / Tg;
    r[M_Tt] = 1.0 / Tt;
    r[M_fwId] = -(m.Edp + (Xqp - Xdp) * m.Iq) / H2;
    r[M_fwIq] = -(m.Eqp + (Xqp - Xdp) * m.Id) / H2;
    r[M_fqId] = -(Xd - Xdp) / Td0p;
    r[M_fdIq] = (Xq - Xqp) / Tq0p;
    r[M_feV] = -KA / TA;
  }
  __syncthreads();
  const int ns = kNsSg * nact - 1;
  const double ws = net.ws;
  bool bad = false;
  const size_t total = (size_t)ns * ns;
  for (size_t e = tid; e < total; e += DYN_THREADS) {
    const int qp = (int)(e % ns), cp = (int)(e / ns);
    const int q = qp + 1, c = cp + 1;          // compact full indices
    const int i = q / kNsSg, sr = q % kNsSg;
    const int j = c / kNsSg, tc = c % kNsSg;
    double val = 0.0;
    if (sr == 0) {
      // relative angle row of machine i (i >= 1): ws (e_omega_i - e_omega_0)
      if (c == kNsSg * i + 1) val += ws;
      if (c == 1) val -= ws;
    } else {
      const double* r = mrec + (size_t)i * M_REC;
      if (j == i) {
        switch (sr * 8 + tc) {
          case 1 * 8 + 1: val = r[M_D1]; break;
          case 1 * 8 + 2: val = r[M_Iq]; break;
          case 1 * 8 + 3: val = r[M_Id]; break;
          case 1 * 8 + 6: val = r[M_H2]; break;
          case 2 * 8 + 2: val = -r[M_Td]; break;
          case 2 * 8 + 4: val = r[M_Td]; break;
          case 3 * 8 + 3: val = -r[M_Tq]; break;
          case 4 * 8 + 4: val = -r[M_TA]; break;
          case 5 * 8 + 1: val = r[M_RTg]; break;
          case 5 * 8 + 5: val = -r[M_Tg]; break;
          case 6 * 8 + 5: val = r[M_Tt]; break;
          case 6 * 8 + 6: val = -r[M_Tt]; break;
          default: break;
        }
      }
      if (tc == 0 || tc == 2 || tc == 3) {
        const int gi = gl[i], gj = gl[j];
        const int m = (tc == 0) ? 0 : (tc == 2 ? 1 : 2);
        // X = g_y^{-1} g_x sits in columns ny.. of the row-major system
        const double* X = K + ny + 3 * gj + m;
#define XR(row) X[(size_t)(row) * ldy]
        switch (sr) {
          case 1: val -= r[M_fwId] * XR(gi) + r[M_fwIq] * XR(ng + gi); break;
          case 2: val -= r[M_fqId] * XR(gi); break;
          case 3: val -= r[M_fdIq] * XR(ng + gi); break;
          case 4: val -= r[M_feV] * XR(2 * ng + nb + net.gen_bus[gi]); break;
          default: break;
        }
#undef XR
      }
    }
    bad |= !__builtin_isfinite(val);
    A[(size_t)cp * lda + qp] = val;
  }
  if (bad) s_bad = 1;            // benign race: every writer stores 1
  __syncthreads();
  if (tid == 0) {
    S.n_states = ns;
    S.job = 0;
    if (s_bad) {
      S.cause |= C_NUMERICAL;
      S.phase = PH_FIN;
    } else {
      S.phase = PH_EIG;
    }
  }
}

void launch_dyn_assemble(const DevNet& net, const Slots& s, int count, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_dyn_assemble, dim3(count), dim3(DYN_THREADS), 0, st, net, s, count);
}

size_t form_state_lds(int ng) {
  return sizeof(double) * (size_t)ng * 15 + sizeof(int) * (size_t)ng + 16;
}

void dyn_set_attrs(size_t bytes) {
  hipFuncSetAttribute(reinterpret_cast<const void*>(k_form_state),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

void launch_form_state(const DevNet& net, const Slots& s, int count, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_form_state, dim3(count), dim3(DYN_THREADS), form_state_lds(net.ng),
                     st, net, s, count);
}

}  // namespace cs
