// Power at one end of a pi branch in polar coordinates, with derivatives.
//
// For the end with own bus o and other bus r, theta = th_o - th_r:
//   A = g_or cos(theta) + b_or sin(theta),  B = g_or sin(theta) - b_or cos(theta)
//   P = V_o^2 g_oo + V_o V_r A
//   Q = -V_o^2 b_oo + V_o V_r B
// (from S_o = V_o conj(Y_oo V_o + Y_or V_r)).  dA/dtheta = -B, dB/dtheta = A.
// Gradients and Hessians are over (th_o, th_r, V_o, V_r); Hessians are packed
// symmetric 4x4: [00 01 02 03 11 12 13 22 23 33].
#pragma once
#include <hip/hip_runtime.h>

namespace cs {

struct EndPower {
  double P, Q;
  double dP[4], dQ[4];
  double A, B;
};

__device__ inline void end_power(double vo, double vr, double th, double goo,
                                 double boo, double gor, double bor,
                                 EndPower& e) {
  double s, c;
  sincos(th, &s, &c);
  const double A = gor * c + bor * s;
  const double B = gor * s - bor * c;
  const double vv = vo * vr;
  e.A = A;
  e.B = B;
  e.P = vo * vo * goo + vv * A;
  e.Q = -vo * vo * boo + vv * B;
  e.dP[0] = -vv * B;
  e.dP[1] = vv * B;
  e.dP[2] = 2.0 * vo * goo + vr * A;
  e.dP[3] = vo * A;
  e.dQ[0] = vv * A;
  e.dQ[1] = -vv * A;
  e.dQ[2] = -2.0 * vo * boo + vr * B;
  e.dQ[3] = vo * B;
}

// Hessians of P and Q at one end, packed, own ordering.
__device__ inline void end_hessians(double vo, double vr, double goo, double boo,
                                    const EndPower& e, double* HP, double* HQ) {
  const double vv = vo * vr, A = e.A, B = e.B;
  HP[0] = -vv * A; HP[1] = vv * A; HP[2] = -vr * B; HP[3] = -vo * B;
  HP[4] = -vv * A; HP[5] = vr * B; HP[6] = vo * B;
  HP[7] = 2.0 * goo; HP[8] = A; HP[9] = 0.0;
  HQ[0] = -vv * B; HQ[1] = vv * B; HQ[2] = vr * A; HQ[3] = vo * A;
  HQ[4] = -vv * B; HQ[5] = -vr * A; HQ[6] = -vo * A;
  HQ[7] = -2.0 * boo; HQ[8] = B; HQ[9] = 0.0;
}

__device__ inline int pk(int i, int j) {  // packed index of (i, j), i, j < 4
  if (i > j) { int t = i; i = j; j = t; }
  // rows: 0 -> 0..3, 1 -> 4..6, 2 -> 7..8, 3 -> 9
  const int base[4] = {0, 4, 7, 9};
  return base[i] + (j - i);
}

}  // namespace cs
