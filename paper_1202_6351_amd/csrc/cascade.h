// cascade.h -- per-node arithmetic of the cascaded (central-moment) D2Q9
// collision with central-moment forcing, and its reverse (transposed
// Jacobian), for gfx950.
//
// What is computed (Ning & Premnath, Section II): with rho = sum f-bar and
// u = (sum f-bar e + F/2)/rho, the central moments
// C_mn = sum_a f-bar_a (e_ax - u_x)^m (e_ay - u_y)^n are relaxed each at its
// own rate towards the transformed attractors (Sec. II, the kappa-bar^eq
// list; the explicit collision kernels g3..g8 plus the source S reach
// exactly this), the first-order ones going from -F/2 to +F/2 (the source's
// central moments are (0, F_x, F_y, 0, ...)):
//   C*_00 = rho, C*_10 = F_x/2, C*_01 = F_y/2,
//   (C_20 + C_02)* = (C_20 + C_02) + w3 (2 rho/3 - (C_20 + C_02)),
//   (C_20 - C_02)* = (1 - w4)(C_20 - C_02),  C*_11 = (1 - w5) C_11,
//   C*_21 = (1 - w6) C_21,  C*_12 = (1 - w7) C_12,
//   C*_22 = C_22 + w8 (rho/9 - C_22),
// and f~-bar is the D2Q9 vector with those central moments.
//
// How (differs from the paper's route, same result): D2Q9 is the tensor
// product of {-1, 0, +1} with itself, so the monomial-moment transform, the
// binomial shift to central moments (Sec. II binomial formula) and their
// inverses all factor into 3-point operations along x then y.  Everything is
// written for the deviation d = f-bar - w rho0 from the rest equilibrium:
// the rest part's raw moments rho0 (1,0,1/3) x (1,0,1/3) map to the central
// moments rho0 Cw(u) with Cw = (1, -u, 1/3 + u^2) per axis, so the
// relaxation can be carried out on Delta C = C - rho0 Cw whose every term is
// of order |u| or rho - rho0.  No O(1) quantity is ever cancelled, which is
// what lets FP32 arithmetic and 16-bit storage hold small velocities.
//
// The collision is applied as an increment, as the paper writes it
// (f~-bar = f-bar + K g + S): Delta C = C* - C is formed in central-moment
// space (its conserved part is exactly (0, F_x, F_y)), shifted back to raw
// moments and inverted, and only then added to the incoming d.  Rounding in
// the transforms is then relative to the small non-equilibrium change, not
// to d itself; with the full post-collision moments instead, FP32 rounding
// in the inverse transform repeats identically every step of a steady flow
// and acts as a spurious body force (measured: 7e-5 relative velocity error
// on a 256 x 64 Poiseuille channel after 4000 steps, against 1e-7 with the
// increment).
#pragma once

#include <hip/hip_runtime.h>

// Every per-node function is host-callable too, so the arithmetic can be
// unit-tested on the CPU (FP64 instantiation) against the reference.
#define LBM_HD __host__ __device__ __forceinline__

namespace lbm {

// Direction order of Section II.  DIR[J][I] is the direction with
// e_x = I - 1, e_y = J - 1.
constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr int DIR[3][3] = {{7, 4, 8}, {3, 0, 1}, {6, 2, 5}};

template <typename R>
struct Rates {
  R w3, w4, w5, w6, w7, w8;        // relaxation rates omega_3..omega_8
  R hw3, hw4, w5x2;                // omega_3 / 2, omega_4 / 2, 2 omega_5 (exact scalings)
  R rho0;                          // reference density of the deviations
};

template <typename R>
LBM_HD Rates<R> make_rates(const R w[6], R rho0) {
  Rates<R> r;
  r.w3 = w[0]; r.w4 = w[1]; r.w5 = w[2]; r.w6 = w[3]; r.w7 = w[4]; r.w8 = w[5];
  r.hw3 = R(0.5) * r.w3;
  r.hw4 = R(0.5) * r.w4;
  r.w5x2 = R(2) * r.w5;
  r.rho0 = rho0;
  return r;
}

// a * b + c rounded once.  Every fused multiply-add of the step's collision
// is written out, so its rounding is fixed by the source and identical in
// every kernel the collision is inlined into.
LBM_HD float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
LBM_HD double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ------------------------------------------------------ 3-point operators
// Moments of (p-, p0, p+) on {-1, 0, +1}: m0 = sum, m1 = p+ - p-, m2 = p+ + p-.
template <typename R>
LBM_HD void ax_mom(R pm, R p0, R pp, R& m0, R& m1, R& m2) {
  m2 = pp + pm;
  m1 = pp - pm;
  m0 = m2 + p0;
}
template <typename R>
LBM_HD void ax_mom_T(R a0, R a1, R a2, R& apm, R& ap0, R& app) {
  const R s = a0 + a2;
  ap0 = a0;
  apm = s - a1;
  app = s + a1;
}
// Inverse: p0 = m0 - m2, p-+ = (m2 -+ m1)/2.
template <typename R>
LBM_HD void ax_inv(R m0, R m1, R m2, R& pm, R& p0, R& pp) {
  p0 = m0 - m2;
  pm = R(0.5) * (m2 - m1);
  pp = R(0.5) * (m2 + m1);
}
template <typename R>
LBM_HD void ax_inv_T(R apm, R ap0, R app, R& a0, R& a1, R& a2) {
  a0 = ap0;
  a1 = R(0.5) * (app - apm);
  a2 = R(0.5) * (app + apm) - ap0;
}
// Shift raw -> central about u: c1 = m1 - u m0, c2 = m2 - 2u m1 + u^2 m0.
template <typename R>
LBM_HD void ax_ctr(R u, R m0, R m1, R m2, R& c0, R& c1, R& c2) {
  c0 = m0;
  c1 = m1 - u * m0;
  c2 = m2 - u * (m1 + c1);
}
// Transpose of ax_ctr at inputs (m0, m1, m2); accumulates d/du into au.
template <typename R>
LBM_HD void ax_ctr_T(R u, R m0, R m1, R a0, R a1, R a2,
                                         R& am0, R& am1, R& am2, R& au) {
  const R c1 = m1 - u * m0;
  am2 = a2;
  am1 = a1 - R(2) * u * a2;
  am0 = a0 - u * (a1 - u * a2);
  au += -m0 * a1 - R(2) * c1 * a2;
}
// Shift central -> raw about u: m1 = c1 + u c0, m2 = c2 + 2u c1 + u^2 c0.
template <typename R>
LBM_HD void ax_unc(R u, R c0, R c1, R c2, R& m0, R& m1, R& m2) {
  m0 = c0;
  m1 = c1 + u * c0;
  m2 = c2 + u * (c1 + m1);
}
template <typename R>
LBM_HD void ax_unc_T(R u, R c0, R c1, R a0, R a1, R a2,
                                         R& ac0, R& ac1, R& ac2, R& au) {
  const R m1 = c1 + u * c0;
  ac2 = a2;
  ac1 = a1 + R(2) * u * a2;
  ac0 = a0 + u * (a1 + u * a2);
  au += c0 * a1 + R(2) * m1 * a2;
}

// --------------------------------------------------------------- relaxation
// Transformed equilibrium of Sec. II in deviation form: central moments
// (rho, hFx, hFy, rho/3, rho/3, 0, 0, 0, rho/9) about u minus rho0 Cw(u).
// With hF = -F/2 this is f^eq - S/2 (the initial state); its entries of
// order >= 2 are the relaxation targets of the collision.
template <typename R>
LBM_HD void equilibrium_cm(R r0, R drho, R ux, R uy, R hFx, R hFy, R Cs[3][3]) {
  const R ux2 = ux * ux, uy2 = uy * uy;
  Cs[0][0] = drho;
  Cs[1][0] = hFx + r0 * ux;
  Cs[0][1] = hFy + r0 * uy;
  Cs[2][0] = R(1.0 / 3.0) * drho - r0 * ux2;
  Cs[0][2] = R(1.0 / 3.0) * drho - r0 * uy2;
  Cs[1][1] = -r0 * (ux * uy);
  Cs[2][1] = r0 * uy * (R(1.0 / 3.0) + ux2);
  Cs[1][2] = r0 * ux * (R(1.0 / 3.0) + uy2);
  Cs[2][2] = R(1.0 / 9.0) * drho - r0 * (R(1.0 / 3.0) * (ux2 + uy2) + ux2 * uy2);
}

template <typename R>
LBM_HD void equilibrium_cm_T(R r0, R ux, R uy, const R aCs[3][3], R& adrho,
                                                 R& aux, R& auy, R& ahFx, R& ahFy) {
  const R ux2 = ux * ux, uy2 = uy * uy;
  adrho += aCs[0][0] + R(1.0 / 3.0) * (aCs[2][0] + aCs[0][2]) + R(1.0 / 9.0) * aCs[2][2];
  ahFx += aCs[1][0];
  ahFy += aCs[0][1];
  // d/du_x of the entries, the terms that carry a factor u_x gathered in gx
  // (and likewise for u_y):
  //   d/du_x = r0 [aCs10 - u_y aCs11 + (1/3 + u_y^2) aCs12
  //                + u_x (2 (u_y aCs21 - aCs20) - (2/3 + 2 u_y^2) aCs22)]
  const R gx = fmad(-fmad(R(2), uy2, R(2.0 / 3.0)), aCs[2][2], R(2) * fmad(uy, aCs[2][1], -aCs[2][0]));
  const R gy = fmad(-fmad(R(2), ux2, R(2.0 / 3.0)), aCs[2][2], R(2) * fmad(ux, aCs[1][2], -aCs[0][2]));
  aux = fmad(r0, fmad(ux, gx, fmad(-uy, aCs[1][1], fmad(R(1.0 / 3.0) + uy2, aCs[1][2], aCs[1][0]))), aux);
  auy = fmad(r0, fmad(uy, gy, fmad(-ux, aCs[1][1], fmad(R(1.0 / 3.0) + ux2, aCs[2][1], aCs[0][1]))), auy);
}

// ------------------------------------------------------------ node passes
// Raw moments of a node's d (x then y).
template <typename R>
LBM_HD void raw_moments(const R d[9], R M[3][3]) {
  R A[3][3];  // A[J][m]
#pragma unroll
  for (int J = 0; J < 3; ++J) ax_mom(d[DIR[J][0]], d[DIR[J][1]], d[DIR[J][2]], A[J][0], A[J][1], A[J][2]);
#pragma unroll
  for (int m = 0; m < 3; ++m) ax_mom(A[0][m], A[1][m], A[2][m], M[m][0], M[m][1], M[m][2]);
}

// Central moments (deviation form) Delta C about u from raw moments M;
// X receives the intermediate after the x shift.
template <typename R>
LBM_HD void central(R ux, R uy, const R M[3][3], R X[3][3], R C[3][3]) {
#pragma unroll
  for (int n = 0; n < 3; ++n) ax_ctr(ux, M[0][n], M[1][n], M[2][n], X[0][n], X[1][n], X[2][n]);
#pragma unroll
  for (int m = 0; m < 3; ++m) ax_ctr(uy, X[m][0], X[m][1], X[m][2], C[m][0], C[m][1], C[m][2]);
}

// Populations (deviation form) with central moments Cs about u; Y receives
// the intermediate after the y shift.  Linear in Cs: also maps a change of
// central moments to the change of populations.
template <typename R>
LBM_HD void populations(R ux, R uy, const R Cs[3][3], R Y[3][3], R out[9]) {
  R Mo[3][3];
#pragma unroll
  for (int m = 0; m < 3; ++m) ax_unc(uy, Cs[m][0], Cs[m][1], Cs[m][2], Y[m][0], Y[m][1], Y[m][2]);
#pragma unroll
  for (int n = 0; n < 3; ++n) ax_unc(ux, Y[0][n], Y[1][n], Y[2][n], Mo[0][n], Mo[1][n], Mo[2][n]);
  R B[3][3];  // B[J][m]
#pragma unroll
  for (int m = 0; m < 3; ++m) ax_inv(Mo[m][0], Mo[m][1], Mo[m][2], B[0][m], B[1][m], B[2][m]);
#pragma unroll
  for (int J = 0; J < 3; ++J)
    ax_inv(B[J][0], B[J][1], B[J][2], out[DIR[J][0]], out[DIR[J][1]], out[DIR[J][2]]);
}

// Reverse of populations(): cotangent aout of the output -> aCs; accumulates
// d/du into aux, auy.
template <typename R>
LBM_HD void populations_T(R ux, R uy, const R Cs[3][3], const R Y[3][3],
                                              const R aout[9], R aCs[3][3], R& aux, R& auy) {
  R aB[3][3];
#pragma unroll
  for (int J = 0; J < 3; ++J)
    ax_inv_T(aout[DIR[J][0]], aout[DIR[J][1]], aout[DIR[J][2]], aB[J][0], aB[J][1], aB[J][2]);
  R aMo[3][3];
#pragma unroll
  for (int m = 0; m < 3; ++m) ax_inv_T(aB[0][m], aB[1][m], aB[2][m], aMo[m][0], aMo[m][1], aMo[m][2]);
  R aY[3][3];
#pragma unroll
  for (int n = 0; n < 3; ++n)
    ax_unc_T(ux, Y[0][n], Y[1][n], aMo[0][n], aMo[1][n], aMo[2][n], aY[0][n], aY[1][n], aY[2][n], aux);
#pragma unroll
  for (int m = 0; m < 3; ++m)
    ax_unc_T(uy, Cs[m][0], Cs[m][1], aY[m][0], aY[m][1], aY[m][2], aCs[m][0], aCs[m][1], aCs[m][2], auy);
}

// Reciprocal: IEEE division in double; for float the hardware estimate
// (v_rcp_f32, within 1 ulp) instead of the correctly rounded division
// sequence.
LBM_HD double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// Hydrodynamic fields from the raw moments of d (Sec. II): rho = rho0 +
// M_00, u = (M_10 + F_x/2, M_01 + F_y/2)/rho (the rest part has no momentum).
template <typename R>
LBM_HD void node_fields(const Rates<R>& r, const R M[3][3], R Fx, R Fy,
                                            R& drho, R& inv_rho, R& ux, R& uy) {
  drho = M[0][0];
  inv_rho = R(1) / (r.rho0 + drho);
  ux = (M[1][0] + R(0.5) * Fx) * inv_rho;
  uy = (M[0][1] + R(0.5) * Fy) * inv_rho;
}

// Transposed Jacobian of the collision at the pre-collision deviations d:
// given the cotangent a of the post-collision deviations, returns the
// cotangent ad of d and adds the force cotangent to aFx, aFy.  The forward
// part recomputes only what the reverse part reads (raw and central moments,
// u, the increments Delta C and their back-shifted values, no post-collision
// populations); the reverse part takes each step of the collision backwards
// (inverse transform, back shift, relaxation with its attractors, shift to
// central moments, hydrodynamic fields, raw moments) and leaves out the terms
// of the structural zeros: Delta C_00 = 0, Delta C_10 = F_x and Delta C_01 =
// F_y (their cotangents go to the force only), and C_00, C_10, C_01 are not
// relaxed (no cotangent reaches them).
template <typename R>
LBM_HD void collide_adj(const Rates<R>& r, R Fx, R Fy, const R d[9], const R a[9], R ad[9], R& aFx, R& aFy) {
  const R r0 = r.rho0, third = R(1.0 / 3.0);
  // ---------------------------------------------------------------- forward
  R M[3][3];
  raw_moments(d, M);
  const R drho = M[0][0];
  const R inv = recip(r0 + drho);
  const R ux = fmad(R(0.5), Fx, M[1][0]) * inv;
  const R uy = fmad(R(0.5), Fy, M[0][1]) * inv;
  R X1[3], X2[3];  // after the x shift: X[1][n], X[2][n] (X[0][n] = M[0][n])
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    X1[n] = fmad(-ux, M[0][n], M[1][n]);
    X2[n] = fmad(-ux, M[1][n] + X1[n], M[2][n]);
  }
  const R C01 = fmad(-uy, M[0][0], M[0][1]);
  const R C02 = fmad(-uy, M[0][1] + C01, M[0][2]);
  const R C11 = fmad(-uy, X1[0], X1[1]);
  const R C12 = fmad(-uy, X1[1] + C11, X1[2]);
  const R C20 = X2[0];
  const R C21 = fmad(-uy, X2[0], X2[1]);
  // (C22 itself is not needed: the step is linear in it)
  const R ux2 = ux * ux, uy2 = uy * uy, uxy = ux * uy;
  const R tx = third + ux2, ty = third + uy2;
  // increments Delta C = omega (E - C) of the relaxed moments (E: the
  // attractors in deviation form), the bulk and shear parts of C20, C02
  // formed as in the step's collision
  const R Es = fmad(-r0, ux2 + uy2, fmad(R(2.0 / 3.0), drho, -(C20 + C02)));
  const R dd2 = r.hw4 * fmad(-r0, ux2 - uy2, -(C20 - C02));
  const R D20 = fmad(r.hw3, Es, dd2), D02 = fmad(r.hw3, Es, -dd2);
  const R D11 = r.w5 * fmad(-r0, uxy, -C11);
  const R D21 = r.w6 * fmad(r0 * uy, tx, -C21);
  const R D12 = r.w7 * fmad(r0 * ux, ty, -C12);
  // back shift by +u (y, then x): the values whose cotangents carry u
  const R uy2x = uy + uy, ux2x = ux + ux;
  const R Y02 = fmad(uy2x, Fy, D02);
  const R Y11 = fmad(uy, Fx, D11);
  const R Y12 = fmad(uy, D11 + Y11, D12);
  const R Y21 = fmad(uy, D20, D21);
  const R Mo11 = fmad(ux, Fy, Y11);
  const R Mo12 = fmad(ux, Y02, Y12);
  // ---------------------------------------------------------------- reverse
  // inverse transform (x rows, then y), transposed
  R aB[3][3], aMo[3][3];
#pragma unroll
  for (int J = 0; J < 3; ++J) ax_inv_T(a[DIR[J][0]], a[DIR[J][1]], a[DIR[J][2]], aB[J][0], aB[J][1], aB[J][2]);
#pragma unroll
  for (int m = 0; m < 3; ++m) ax_inv_T(aB[0][m], aB[1][m], aB[2][m], aMo[m][0], aMo[m][1], aMo[m][2]);
  // x shift by +ux, transposed; the shifted column n = 0 is (0, F_x, .),
  // n = 1 is (F_y, Mo11, .), n = 2 is (Y02, Mo12, .)
  R aY[3][3];
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    aY[2][n] = aMo[2][n];
    aY[1][n] = fmad(ux2x, aMo[2][n], aMo[1][n]);
    aY[0][n] = fmad(ux, fmad(ux, aMo[2][n], aMo[1][n]), aMo[0][n]);
  }
  // the u_x cotangent: hx collects the terms with a factor 2 (added twice
  // at the end), aux the others; likewise hy and auy for u_y
  R hx = Fx * aMo[2][0];
  hx = fmad(Mo11, aMo[2][1], hx);
  hx = fmad(Mo12, aMo[2][2], hx);
  R aux = fmad(Y02, aMo[1][2], Fy * aMo[1][1]);
  // y shift by +uy, transposed, per row m (Delta C_m0, Delta C_m1, Delta C_m2)
  const R aD02 = aY[0][2], aD01 = fmad(uy2x, aY[0][2], aY[0][1]);
  const R aD12 = aY[1][2], aD11 = fmad(uy2x, aY[1][2], aY[1][1]);
  const R aD10 = fmad(uy, fmad(uy, aY[1][2], aY[1][1]), aY[1][0]);
  const R aD22 = aY[2][2], aD21 = fmad(uy2x, aY[2][2], aY[2][1]);
  const R aD20 = fmad(uy, fmad(uy, aY[2][2], aY[2][1]), aY[2][0]);
  R hy = Fy * aY[0][2];
  hy = fmad(Y11, aY[1][2], hy);
  hy = fmad(Y21, aY[2][2], hy);
  R auy = fmad(D20, aY[2][1], Fx * aY[1][1]);
  aFx += aD10;
  aFy += aD01;
  // relaxation, transposed: the cotangents of E - C per relaxed moment
  const R as = r.hw3 * (aD20 + aD02), adv = r.hw4 * (aD20 - aD02);
  const R a11 = r.w5 * aD11, a21 = r.w6 * aD21, a12 = r.w7 * aD12, a22 = r.w8 * aD22;
  const R aC20 = -(as + adv), aC02 = adv - as;
  R adrho = fmad(R(2.0 / 3.0), as, R(1.0 / 9.0) * a22);
  // attractors: d/d(u_x^2), d/d(u_y^2), d/d(u_x u_y), then the chain to u
  // (as + adv = -aC20, as - adv = -aC02)
  const R aux2 = fmad(-r0, fmad(ty, a22, -aC20), r0 * uy * a21);
  const R auy2 = fmad(-r0, fmad(tx, a22, -aC02), r0 * ux * a12);
  const R auxy = -r0 * a11;
  aux = fmad(ux2x, aux2, fmad(uy, auxy, fmad(r0 * ty, a12, aux)));
  auy = fmad(uy2x, auy2, fmad(ux, auxy, fmad(r0 * tx, a21, auy)));
  // y shift to central moments, transposed (aC_00 = aC_10 = aC_01 = 0; the
  // cotangents of C_11, C_21, C_12, C_22 are -a11, -a21, -a12, -a22)
  const R aX02 = aC02, aX01 = -uy2x * aC02, aX00 = uy2 * aC02;
  const R aX12 = -a12, aX11 = fmad(uy2x, a12, -a11);
  const R aX10 = -uy * fmad(uy, a12, -a11);
  const R aX22 = -a22, aX21 = fmad(uy2x, a22, -a21);
  const R aX20 = fmad(-uy, fmad(uy, a22, -a21), aC20);
  hy = fmad(-C01, aC02, hy);
  hy = fmad(C11, a12, hy);
  hy = fmad(C21, a22, hy);
  auy = fmad(X1[0], a11, auy);
  auy = fmad(X2[0], a21, auy);
  // x shift to central moments, transposed, per column n
  const R aXc[3][3] = {{aX00, aX01, aX02}, {aX10, aX11, aX12}, {aX20, aX21, aX22}};
  R aM[3][3];
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    aM[2][n] = aXc[2][n];
    aM[1][n] = fmad(-ux2x, aXc[2][n], aXc[1][n]);
    aM[0][n] = fmad(-ux, fmad(-ux, aXc[2][n], aXc[1][n]), aXc[0][n]);
    aux = fmad(-M[0][n], aXc[1][n], aux);
    hx = fmad(-X1[n], aXc[2][n], hx);
  }
  aux = fmad(R(2), hx, aux);
  auy = fmad(R(2), hy, auy);
  // u = (M_10 + F_x/2, M_01 + F_y/2) / (rho0 + M_00)
  const R ajx = aux * inv, ajy = auy * inv;
  aM[0][0] = fmad(-ajx, ux, fmad(-ajy, uy, aM[0][0] + adrho));
  aM[1][0] += ajx;
  aM[0][1] += ajy;
  aFx = fmad(R(0.5), ajx, aFx);
  aFy = fmad(R(0.5), ajy, aFy);
  // raw moments, transposed; the identity path adds a
  R aA[3][3];
#pragma unroll
  for (int m = 0; m < 3; ++m) ax_mom_T(aM[m][0], aM[m][1], aM[m][2], aA[0][m], aA[1][m], aA[2][m]);
#pragma unroll
  for (int J = 0; J < 3; ++J) {
    R a0, a1, a2;
    ax_mom_T(aA[J][0], aA[J][1], aA[J][2], a0, a1, a2);
    ad[DIR[J][0]] = a[DIR[J][0]] + a0;
    ad[DIR[J][1]] = a[DIR[J][1]] + a1;
    ad[DIR[J][2]] = a[DIR[J][2]] + a2;
  }
}

// The collision of the step kernels, in the fewest operations: raw moments,
// the fields, central moments (shift in x, then y), the increments Delta C =
// omega (E - C) of the relaxed moments, back shift and inverse transform
// added to d.  Simplifications, all exact in real arithmetic: Delta C_00 =
// 0 and, without a body force, Delta C_10 = Delta C_01 = 0, so those terms
// are dropped; without a body force the
// first-order central moments of d are rho0 u, which stand in for the
// products rho0 u_x, rho0 u_y of the attractors; the 2 Delta C_11, and
// twice the outer rows of the y inverse, are carried so that the factors 1/2
// and 1/4 of the inverse fold into the final multiply-adds.  kUnit678: the
// caller knows omega_6 = omega_7 = omega_8 = 1 (the paper's default), so
// their multiplies, exact identities then, are left out.
template <typename R, bool kForce, bool kUnit678 = false>
LBM_HD void collide_step(const Rates<R>& r, R Fx, R Fy, const R d[9], R out[9]) {
  R M[3][3];
  raw_moments(d, M);
  const R drho = M[0][0];
  const R inv = recip(r.rho0 + drho);
  const R ux = (kForce ? fmad(R(0.5), Fx, M[1][0]) : M[1][0]) * inv;
  const R uy = (kForce ? fmad(R(0.5), Fy, M[0][1]) : M[0][1]) * inv;
  // Central moments of d about u: shift in x (X1, X2 per column n), then in y.
  R X1[3], X2[3];
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    X1[n] = fmad(-ux, M[0][n], M[1][n]);
    X2[n] = fmad(-ux, M[1][n] + X1[n], M[2][n]);
  }
  const R C01 = fmad(-uy, M[0][0], M[0][1]);
  const R C02 = fmad(-uy, M[0][1] + C01, M[0][2]);
  const R C11 = fmad(-uy, X1[0], X1[1]);
  const R C12 = fmad(-uy, X1[1] + C11, X1[2]);
  const R C20 = X2[0];
  const R C21 = fmad(-uy, X2[0], X2[1]);
  const R C22 = fmad(-uy, X2[1] + C21, X2[2]);
  const R r0ux = kForce ? r.rho0 * ux : X1[0];  // C_10 = rho0 u_x - F_x / 2
  const R r0uy = kForce ? r.rho0 * uy : C01;
  // Relaxation: Delta C = omega (E - C), E the attractors in deviation form.
  const R ux2 = ux * ux, uy2 = uy * uy, uxy = ux * uy;
  const R q = ux2 + uy2, p = ux2 - uy2;
  const R Es = fmad(-r.rho0, q, fmad(R(2.0 / 3.0), drho, -(C20 + C02)));
  const R ad = r.hw4 * fmad(-r.rho0, p, -(C20 - C02));
  const R D20 = fmad(r.hw3, Es, ad), D02 = fmad(r.hw3, Es, -ad);
  const R E11mC = fmad(-r.rho0, uxy, -C11);
  const R E21mC = fmad(r0uy, ux2 + R(1.0 / 3.0), -C21);
  const R E12mC = fmad(r0ux, uy2 + R(1.0 / 3.0), -C12);
  const R E22mC = fmad(-r.rho0, fmad(q, R(1.0 / 3.0), uxy * uxy), fmad(R(1.0 / 9.0), drho, -C22));
  const R D21 = kUnit678 ? E21mC : r.w6 * E21mC;
  const R D12 = kUnit678 ? E12mC : r.w7 * E12mC;
  const R D22 = kUnit678 ? E22mC : r.w8 * E22mC;
  // Back to raw moments (shift by +u, y then x) and the inverse transform
  // (y then x), added to d.  B0, B2: twice the rows e_y = -1, +1 of the y
  // inverse; B1: the row e_y = 0.
  R B0[3], B1[3], B2[3];
  if constexpr (kForce) {
    const R D11 = r.w5 * E11mC;
    const R Y02 = fmad(uy + uy, Fy, D02);
    const R Y11 = fmad(uy, Fx, D11);
    const R Y12 = fmad(uy, D11 + Y11, D12);
    const R Y21 = fmad(uy, D20, D21);
    const R Y22 = fmad(uy, D21 + Y21, D22);
    const R Mo20 = fmad(ux + ux, Fx, D20);
    const R Mo11 = fmad(ux, Fy, Y11);
    const R Mo21 = fmad(ux, Y11 + Mo11, Y21);
    const R Mo12 = fmad(ux, Y02, Y12);
    const R Mo22 = fmad(ux, Y12 + Mo12, Y22);
    // columns m = 0 (Mo00 = 0, Mo01 = F_y, Mo02 = Y02), 1 (F_x, Mo11, Mo12), 2
    B1[0] = -Y02;        B0[0] = Y02 - Fy;     B2[0] = Y02 + Fy;
    B1[1] = Fx - Mo12;   B0[1] = Mo12 - Mo11;  B2[1] = Mo12 + Mo11;
    B1[2] = Mo20 - Mo22; B0[2] = Mo22 - Mo21;  B2[2] = Mo22 + Mo21;
  } else {
    const R D11x2 = r.w5x2 * E11mC;
    const R Y12 = fmad(uy, D11x2, D12);
    const R Y21 = fmad(uy, D20, D21);
    const R Y22 = fmad(uy, D21 + Y21, D22);
    const R Mo21 = fmad(ux, D11x2, Y21);
    const R Mo12 = fmad(ux, D02, Y12);
    const R Mo22 = fmad(ux, Y12 + Mo12, Y22);
    // columns m = 0 (0, 0, D02), 1 (0, D11, Mo12), 2 (D20, Mo21, Mo22)
    B1[0] = -D02;        B0[0] = D02;                          B2[0] = D02;
    B1[1] = -Mo12;       B0[1] = fmad(R(-0.5), D11x2, Mo12);  B2[1] = fmad(R(0.5), D11x2, Mo12);
    B1[2] = D20 - Mo22;  B0[2] = Mo22 - Mo21;                  B2[2] = Mo22 + Mo21;
  }
  // x inverse per row: p0 = m0 - m2, p-+ = (m2 -+ m1) / 2.
  out[DIR[1][1]] = d[DIR[1][1]] + (B1[0] - B1[2]);
  out[DIR[1][0]] = fmad(R(0.5), B1[2] - B1[1], d[DIR[1][0]]);
  out[DIR[1][2]] = fmad(R(0.5), B1[2] + B1[1], d[DIR[1][2]]);
  out[DIR[0][1]] = fmad(R(0.5), B0[0] - B0[2], d[DIR[0][1]]);
  out[DIR[0][0]] = fmad(R(0.25), B0[2] - B0[1], d[DIR[0][0]]);
  out[DIR[0][2]] = fmad(R(0.25), B0[2] + B0[1], d[DIR[0][2]]);
  out[DIR[2][1]] = fmad(R(0.5), B2[0] - B2[2], d[DIR[2][1]]);
  out[DIR[2][0]] = fmad(R(0.25), B2[2] - B2[1], d[DIR[2][0]]);
  out[DIR[2][2]] = fmad(R(0.25), B2[2] + B2[1], d[DIR[2][2]]);
}

}  // namespace lbm
