// Linearised state matrix at the OPF point (Section II.B.2).
//
// Device models: two-axis synchronous machine (delta, omega, Eq', Ed') with a
// first-order AVR (Efd) and a governor-turbine (Psv, Pm), stator algebraic
// equations; grid-following converter (PLL angle and integrator, current PI
// integrators, L-filter currents, DC-link voltage and its PI integrator) in
// the PLL frame; constant-impedance loads at the OPF voltage, and the network
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
// and of each converter: PLL locked to its bus (theta_p = theta, v_d = V,
// v_q = 0), i_d = Pg / V, i_q = -Qg / V.  A converter has no algebraic
// currents: its Id, Iq positions of y are identity rows; its right-hand-side
// columns are d g / d(theta_p, i_d, i_q).
//
// State order per device, in ascending generator order: a machine's 7
// states [delta, omega, Eq', Ed', Efd, Psv, Pm], a converter's 8
// [theta_p, x_pll, x_id, x_iq, i_d, i_q, v_dc, x_dc]; local state 0 is the
// angle in both.
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
    if (!gen_on[g] || net.gen_kind[g] != 0) { YY(g, g) = 1.0; YY(ng + g, ng + g) = 1.0; continue; }
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
      if (net.gen_kind[g] != 0) {
        // converter injection P = V (i_d cos phi + i_q sin phi),
        // Q = V (i_d sin phi - i_q cos phi), phi = theta - theta_p = 0
        const double i_d = x[2 * nb + g] / vm, i_q = -x[2 * nb + ng + g] / vm;
        pv += i_d;                     // dP/dV
        qv += -i_q;                    // dQ/dV
        pt += vm * i_q;                // dP/dtheta
        qt += vm * i_d;                // dQ/dtheta
        const int c = ny + 3 * g;
        YY(rp, c + 0) = -vm * i_q;     // d/d theta_p
        YY(rq, c + 0) = -vm * i_d;
        YY(rp, c + 1) = vm;            // d/d i_d
        YY(rq, c + 2) = -vm;           // d/d i_q
        continue;
      }
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

// Per-device record of k_form_state (LDS): the device's f_x and f_y
// coefficients.  Machine fields M_*, converter fields C_* share the slots.
enum { M_D1, M_Iq, M_Id, M_H2, M_Td, M_Tq, M_TA, M_RTg, M_Tg, M_Tt,
       M_fwId, M_fwIq, M_fqId, M_fdIq, M_feV, M_REC };
enum { C_WKPP, C_WKIP, C_KPDC, C_KIDC, C_G, C_KPC, C_RF, C_KIC, C_CV, C_VD, C_ID, C_IQ };
constexpr int kMaxStates = 1024 + 1;   // unreduced states per island

struct FormShared {
  const double* rec;   // [ndev][M_REC]
  const int* gl;       // compact device -> generator
  const int* kind;     // compact device -> kind
  const int* off;      // compact device -> first unreduced state, [ndev + 1]
  const int* sdev;     // unreduced state -> compact device
};

// Entry (q, c) of the unreduced A_full = f_x - f_y X, X = g_y^{-1} g_x held in
// the right-hand-side columns of the factorised algebraic system K.
__device__ inline double full_entry(const FormShared& F, const DevNet& net, const double* K,
                                    int ny, int ldy, int q, int c) {
  const int ng = net.ng, nb = net.nb;
  const int i = F.sdev[q], sr = q - F.off[i];
  const int j = F.sdev[c], tc = c - F.off[j];
  const double* r = F.rec + (size_t)i * M_REC;
  const int ki = F.kind[i], kj = F.kind[j];
  double val = 0.0;
  if (j == i) {
    if (ki == 0) {
      switch (sr * 8 + tc) {
        case 0 * 8 + 1: val = net.ws; break;
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
    } else {
      const double g = r[C_G];
      switch (sr * 8 + tc) {
        case 0 * 8 + 0: val = -r[C_WKPP] * r[C_VD]; break;      // dv_q/dtheta_p = -v_d
        case 0 * 8 + 1: val = r[C_WKIP]; break;
        case 1 * 8 + 0: val = -r[C_VD]; break;
        case 2 * 8 + 4: val = -1.0; break;
        case 2 * 8 + 6: val = r[C_KPDC]; break;
        case 2 * 8 + 7: val = r[C_KIDC]; break;
        case 3 * 8 + 5: val = -1.0; break;
        case 4 * 8 + 4: val = -g * (r[C_KPC] + r[C_RF]); break;
        case 4 * 8 + 2: val = g * r[C_KIC]; break;
        case 4 * 8 + 6: val = g * r[C_KPC] * r[C_KPDC]; break;
        case 4 * 8 + 7: val = g * r[C_KPC] * r[C_KIDC]; break;
        case 5 * 8 + 5: val = -g * (r[C_KPC] + r[C_RF]); break;
        case 5 * 8 + 3: val = g * r[C_KIC]; break;
        case 6 * 8 + 0: val = r[C_IQ] * r[C_VD] / r[C_CV]; break;
        case 6 * 8 + 4: val = -r[C_VD] / r[C_CV]; break;
        case 7 * 8 + 6: val = 1.0; break;
        default: break;
      }
    }
  }
  // - f_y X through the three right-hand-side columns of device j
  int m = -1;
  if (kj == 0) m = (tc == 0) ? 0 : (tc == 2) ? 1 : (tc == 3) ? 2 : -1;
  else m = (tc == 0) ? 0 : (tc == 4) ? 1 : (tc == 5) ? 2 : -1;
  if (m >= 0) {
    const int gi = F.gl[i], gj = F.gl[j];
    const int kb = net.gen_bus[gi];
    const double* X = K + ny + 3 * gj + m;
#define XR(row) X[(size_t)(row) * ldy]
    if (ki == 0) {
      switch (sr) {
        case 1: val -= r[M_fwId] * XR(gi) + r[M_fwIq] * XR(ng + gi); break;
        case 2: val -= r[M_fqId] * XR(gi); break;
        case 3: val -= r[M_fdIq] * XR(ng + gi); break;
        case 4: val -= r[M_feV] * XR(2 * ng + nb + kb); break;
        default: break;
      }
    } else {
      // f_y of the PLL rows: d v_q / d theta = v_d (d v_q / dV = 0); of the
      // DC link: d/dV = -i_d / CV, d/dtheta = -i_q v_d / CV
      switch (sr) {
        case 0: val -= r[C_WKPP] * r[C_VD] * XR(2 * ng + kb); break;
        case 1: val -= r[C_VD] * XR(2 * ng + kb); break;
        case 6:
          val += (r[C_ID] * XR(2 * ng + nb + kb) + r[C_IQ] * r[C_VD] * XR(2 * ng + kb)) / r[C_CV];
          break;
        default: break;
      }
    }
#undef XR
  }
  return val;
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
  double* mrec = shd;                                               // [ng][M_REC]
  int* gl = reinterpret_cast<int*>(mrec + (size_t)ng * M_REC);      // [ng]
  int* kind = gl + ng;                                              // [ng]
  int* off = kind + ng;                                             // [ng + 1]
  int* sdev = off + ng + 1;                                         // [kMaxStates]
  __shared__ int s_nact, s_nfull;
  __shared__ int s_bad;
  const double* x = s.x + (size_t)slot * s.nx;
  const uint8_t* gen_on = s.gen_on + (size_t)slot * ng;
  const double* K = s.K + (size_t)slot * s.k_stride;
  double* A = s.A + (size_t)slot * s.a_stride;
  if (tid == 0) {
    int c = 0, o = 0;
    for (int g = 0; g < ng; ++g)
      if (gen_on[g]) {
        gl[c] = g;
        kind[c] = net.gen_kind[g];
        off[c] = o;
        o += kind[c] == 0 ? kNsSg : kNsGfl;
        ++c;
      }
    off[c] = o;
    s_nact = c;
    s_nfull = o;
    s_bad = S.singular;
  }
  __syncthreads();
  const int nact = s_nact, nfull = s_nfull;
  for (int ci = 0; ci < nact; ++ci)
    for (int q = off[ci] + tid; q < off[ci + 1]; q += DYN_THREADS) sdev[q] = ci;
  for (int ci = tid; ci < nact; ci += DYN_THREADS) {
    const int g = gl[ci];
    const double* p = net.dyn + (size_t)g * kDyn;
    double* r = mrec + (size_t)ci * M_REC;
    if (kind[ci] == 0) {
      const Machine m = equilibrium(net, x, g);
      const double H = p[0], D = p[1], Xd = p[2], Xq = p[3], Xdp = p[4], Xqp = p[5];
      const double Td0p = p[6], Tq0p = p[7], KA = p[9], TA = p[10], R = p[11];
      const double Tg = p[12], Tt = p[13];
      const double H2 = 2.0 * H;
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
    } else {
      // converter row: Kpp Kip Kpc Kic Lf Rf Cdc Kpdc Kidc Vdc0
      const int k = net.gen_bus[g];
      const double vm = x[nb + k];
      r[C_WKPP] = net.ws * p[0];
      r[C_WKIP] = net.ws * p[1];
      r[C_KPC] = p[2];
      r[C_KIC] = p[3];
      r[C_G] = net.ws / p[4];
      r[C_RF] = p[5];
      r[C_CV] = p[6] * p[9];
      r[C_KPDC] = p[7];
      r[C_KIDC] = p[8];
      r[C_VD] = vm;
      r[C_ID] = x[2 * nb + g] / vm;
      r[C_IQ] = -x[2 * nb + ng + g] / vm;
    }
  }
  __syncthreads();
  FormShared F{mrec, gl, kind, off, sdev};
  // reduced state q' = q - 1 (state 0, the first device's angle, removed);
  // every other device's angle row minus the removed angle's row
  const int ns = nfull - 1;
  bool bad = false;
  const size_t total = (size_t)ns * ns;
  for (size_t e = tid; e < total; e += DYN_THREADS) {
    const int qp = (int)(e % ns), cp = (int)(e / ns);
    const int q = qp + 1, c = cp + 1;
    double val = full_entry(F, net, K, ny, ldy, q, c);
    if (q == off[sdev[q]]) val -= full_entry(F, net, K, ny, ldy, 0, c);
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
  return sizeof(double) * (size_t)ng * M_REC + sizeof(int) * (3 * (size_t)ng + 1 + kMaxStates) +
         16;
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
