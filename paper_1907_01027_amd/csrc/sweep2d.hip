// Transport sweeps on a uniform 2D Cartesian mesh for gfx950.
//
// Per direction the upwind DG operator L_l (Sec. 2.1, eq-Ljk; L~_00 of Sec. 3.3.2 for
// the reconstructed scheme) is block lower triangular when cells are visited in the
// upwind order of that direction; all directions of one quadrant share that order.
//
// Work decomposition
//   work item  = (quadrant q, strip s of 16 rows), taken from a ticket counter so a
//                strip is only ever waited on by strips that started after it;
//   workgroup  = all direction slots of q for that strip: W waves, each wave covers
//                16 rows x 4 directions (lane = 16 * slot + row);
//   step t     = lane of row r handles column c = t - r (a skewed wavefront), so the
//                cell below (row r-1, column c) was finished by lane r-1 at step t-1
//                and reaches lane r through one DPP row shift; the cell to the left is
//                the lane's own previous result.  Row 0 reads the trace that the strip
//                below wrote to an edge buffer.
//   chunks     = CW steps.  Before a chunk, the strip-below traces it needs are staged
//                in LDS, and every cell it visits has its source reduced (in FP64, once
//                per workgroup) to three coefficients per source moment, so that the
//                source of direction l is a + |Ox| b + |Oy| c (the quadrant fixes the
//                signs of Ox and Oy).  The
//                coefficients of chunk k+1 are loaded while chunk k runs; the step loop
//                touches only registers and LDS.
//   reductions = per-cell sums over directions: over the 4 slots of a wave with two
//                cross-lane swaps, over waves through LDS, written once per cell and
//                quadrant; a combine kernel adds the quadrants.
// Strips publish "columns finished in my top row" every chunk with an agent-scope
// release; consumers acquire before reading.  Progress words carry the launch epoch
// in the high half so they never need clearing.  Every wait is bounded: a stuck wait
// sets an error flag and the kernel still finishes.
#include "internal.h"
#include "sweep_common.h"

namespace lmdg {
namespace {

// Steps per unrolled group (chunks hold a multiple of it): measured on gfx950, two
// FP64 steps per group schedule better than four, FP32 steps the other way round.
template <typename R>
constexpr int step_group() { return sizeof(R) == 8 ? 2 : 4; }

// Per-lane direction constants.
template <typename R>
struct Dir {
  double ox, oy;        // Omega components
  R aox, aoy;           // |Omega_x|, |Omega_y|
  R w;                  // quadrature weight (0 for padding slots)
  R axhy, ayhx;         // |Omega_x| h_y, |Omega_y| h_x  (face measures times |Omega.nu|)
  R oxhy, oyhx;         // Omega_x h_y, Omega_y h_x
  R sx, sy;             // signs of Omega_x, Omega_y
  int idx;              // caller's direction index, -1 for padding
};

// Source layout per scheme: NS source moments, NC staged values per cell
// (sigma_t|K| followed by 5 coefficients per moment), NRAW FP64 inputs per cell.
template <int S>
struct SrcTraits {
  static constexpr int NS = (S == LMDG_SCHEME_STD) ? 4 : 1;
  // sigma_t|K|, 3 source coefficients per moment, and for RLMDG eps sigma_a|K|
  static constexpr int NC = 1 + 3 * NS + (S == LMDG_SCHEME_RLMDG ? 1 : 0);
  static constexpr int NRAW = (S == LMDG_SCHEME_STD) ? 19 : 13;
  static constexpr int MAXC = (S == LMDG_SCHEME_STD) ? 1 : 2;  // staged cells per thread
};

// With the reconstruction variants (VAR, RLMDG only) every cell also stages its upwind
// rule per axis (a_up, a_uu; see cell_rlmdg_var) and loads the cross sections of its
// two upwind neighbours along each axis; cells hand one more trace value downwind
// (their own upwind average).
template <int S, bool VAR>
struct SrcTraitsV : SrcTraits<S> {
  static constexpr int NC = SrcTraits<S>::NC + (VAR ? 4 : 0);
  static constexpr int NRAW = SrcTraits<S>::NRAW + (VAR ? 8 : 0);
  static constexpr int NF = SchemeTraits<S>::NF + (VAR ? 1 : 0);
};

// ---------------------------------------------------------------- local solves
// Low-memory sweep (L_00 of Sec. 3.2): one unknown per cell and direction.
// Row "test with the cell constant" of eq-Ljk:
//   sigma_t|K| psi + |Ox| h_y (psi - psi_left) + |Oy| h_x (psi - psi_down) = src,
// solved with inv = 1 / (sigma_t|K| + |Ox| h_y + |Oy| h_x), which does not depend on the
// upwind values.  Reductions: w psi (P_0), w Ox h_y (psi_left - psi), w Oy h_x
// (psi_down - psi) (rows xi, eta of Sigma L_10; its xi*eta row vanishes).
template <typename R>
__device__ __forceinline__ void cell_lmdg(const Dir<R>& d, R src, R inv, const R* xin, const R* ydn, R* xo, R* yo,
                                          R* o, R& psi_out) {
  const R psi = (src + d.axhy * xin[0] + d.ayhx * ydn[0]) * inv;
  xo[0] = psi;
  yo[0] = psi;
  o[0] = d.w * psi;
  o[1] = d.w * d.oxhy * (xin[0] - psi);
  o[2] = d.w * d.oyhx * (ydn[0] - psi);
  psi_out = psi;
}

// Reconstructed sweep (L~_00 = L_00 + L_01 R, Sec. 3.3): the cell function in
// direction l is psi + c_xi xi + c_eta eta with upwind slopes (Sec. 3.3.1)
//   c_xi = sign(Ox) k_x (psi - psi_left),  k = 1/2 inside, 1 in the inflow cell
// (where the upwind value is the inflow datum: zero for vacuum, the midpoint value of
// alpha otherwise).  inv = 1 / (sigma_t|K| + |Ox| h_y (1 + k_x) + |Oy| h_x (1 + k_y)).
// A face hands downwind its trace average T, its linear coefficient along the face,
// and the cell average.  Reductions: w psi; the xi / eta / xi*eta rows of
// w (L_10 + L_11 R) applied to the cell function minus the scattering part w M_1 R of
// the second block row G = Sigma (L_10 + L_11 R) - Sigma M_1 P_1 R (the slope mass
// term of L_11 R carries sigma_t |K| / 3, that of M_1 P_1 R (sigma_s/eps) |K| / 3, so
// per direction they combine to eps sigma_a |K| / 3 = aA3: the O(sigma_s/eps) parts
// cancel before any rounding instead of after the direction sum); and w c_xi,
// w c_eta (for P_1 R).
template <typename R>
__device__ __forceinline__ void cell_rlmdg(const Dir<R>& d, R src, R aA3, R inv, R kx, R ky, const R* xin,
                                           const R* ydn, R* xo, R* yo, R* o, R& psi_out) {
  // xin = (T_x of left cell, its c_eta, its average); ydn = (T_y, c_xi, average) of cell below
  const R third = R(1) / R(3);
  const R psi = (src + d.axhy * (xin[0] + kx * xin[2]) + d.ayhx * (ydn[0] + ky * ydn[2])) * inv;
  const R cxi = d.sx * kx * (psi - xin[2]);
  const R ceta = d.sy * ky * (psi - ydn[2]);
  xo[0] = psi + kx * (psi - xin[2]);
  xo[1] = ceta;
  xo[2] = psi;
  yo[0] = psi + ky * (psi - ydn[2]);
  yo[1] = cxi;
  yo[2] = psi;
  o[0] = d.w * psi;
  o[1] = d.w * (d.oxhy * (xin[0] - psi) + (aA3 + d.axhy + d.ayhx * third) * cxi - d.ayhx * third * ydn[1]);
  o[2] = d.w * (d.oyhx * (ydn[0] - psi) + (aA3 + d.ayhx + d.axhy * third) * ceta - d.axhy * third * xin[1]);
  o[3] = d.w * third * (d.oxhy * (xin[1] - ceta) + d.oyhx * (ydn[1] - cxi));
  o[4] = d.w * cxi;
  o[5] = d.w * ceta;
  psi_out = psi;
}

// Reconstructed sweep with a per-cell upwind rule (the reconstruction variants): along
// each axis the slope is c = s (k psi - a_up psi_up + a_uu psi_upup) with k = a_up - a_uu
// (constants have no slope): (a_up, a_uu) = (1, 0) in the inflow cell (psi_up the
// inflow value), (1/2, 0) for the two-cell difference, (1, 1/4) for the three-cell
// quadratic (3 psi - 4 psi_up + psi_upup) / 4, (0, 0) where the reconstruction is
// suppressed.  Traces handed downwind: (outflow face average, linear coefficient along
// the face, cell average, the cell's own upwind average along that axis).
// adj: the adjoint sweep of the reconstructed scheme (rules k = 1 in the outflow cell,
// 1/2 elsewhere; see adj_rlm_source_kernel), whose reductions are those of the
// low-memory scheme, w psi and w Sigma L_10 psi (rows xi, eta), the other rows zero.
template <typename R>
__device__ __forceinline__ void cell_rlmdg_var(const Dir<R>& d, R src, R aA3, R inv, const R* ru, const R* xin,
                                               const R* ydn, R* xo, R* yo, R* o, R& psi_out, bool adj) {
  const R third = R(1) / R(3);
  const R psi = (src + d.axhy * (xin[0] + ru[0] * xin[2] - ru[1] * xin[3]) +
                 d.ayhx * (ydn[0] + ru[2] * ydn[2] - ru[3] * ydn[3])) *
                inv;
  const R dx = (ru[0] - ru[1]) * psi - ru[0] * xin[2] + ru[1] * xin[3];  // = s_x c_xi
  const R dy = (ru[2] - ru[3]) * psi - ru[2] * ydn[2] + ru[3] * ydn[3];
  const R cxi = d.sx * dx;
  const R ceta = d.sy * dy;
  xo[0] = psi + dx;
  xo[1] = ceta;
  xo[2] = psi;
  xo[3] = xin[2];
  yo[0] = psi + dy;
  yo[1] = cxi;
  yo[2] = psi;
  yo[3] = ydn[2];
  o[0] = d.w * psi;
  if (adj) {
    o[1] = d.w * d.oxhy * (xin[2] - psi);
    o[2] = d.w * d.oyhx * (ydn[2] - psi);
    o[3] = o[4] = o[5] = R(0);
  } else {
    o[1] = d.w * (d.oxhy * (xin[0] - psi) + (aA3 + d.axhy + d.ayhx * third) * cxi - d.ayhx * third * ydn[1]);
    o[2] = d.w * (d.oyhx * (ydn[0] - psi) + (aA3 + d.ayhx + d.axhy * third) * ceta - d.axhy * third * xin[1]);
    o[3] = d.w * third * (d.oxhy * (xin[1] - ceta) + d.oyhx * (ydn[1] - cxi));
    o[4] = d.w * cxi;
    o[5] = d.w * ceta;
  }
  psi_out = psi;
}

// Local block (coef M + streaming + outflow faces) of the standard sweep.
// ax = |Ox| h_y, ay = |Oy| h_x, oxhy = Ox h_y, oyhx = Oy h_x, sx/sy the signs.
template <typename T>
__device__ __forceinline__ void std_block(T coef, T ax, T ay, T oxhy, T oyhx, T sx, T sy, T m[4][4]) {
  const T third = T(1) / T(3), ninth = T(1) / T(9);
  // mass
  m[0][0] = coef;           m[0][1] = 0;              m[0][2] = 0;              m[0][3] = 0;
  m[1][0] = 0;              m[1][1] = coef * third;   m[1][2] = 0;              m[1][3] = 0;
  m[2][0] = 0;              m[2][1] = 0;              m[2][2] = coef * third;   m[2][3] = 0;
  m[3][0] = 0;              m[3][1] = 0;              m[3][2] = 0;              m[3][3] = coef * ninth;
  // -int u Omega.grad v (rows = test function)
  m[1][0] += -T(2) * oxhy;
  m[2][0] += -T(2) * oyhx;
  m[3][2] += -T(2) * third * oxhy;
  m[3][1] += -T(2) * third * oyhx;
  // outflow face xi = sx: trace (c0 + sx c1) + (c2 + sx c3) eta
  m[0][0] += ax;       m[0][1] += ax * sx;
  m[1][0] += ax * sx;  m[1][1] += ax;
  m[2][2] += ax * third;      m[2][3] += ax * sx * third;
  m[3][2] += ax * sx * third; m[3][3] += ax * third;
  // outflow face eta = sy: trace (c0 + sy c2) + (c1 + sy c3) xi
  m[0][0] += ay;       m[0][2] += ay * sy;
  m[2][0] += ay * sy;  m[2][2] += ay;
  m[1][1] += ay * third;      m[1][3] += ay * sy * third;
  m[3][1] += ay * sy * third; m[3][3] += ay * third;
}

// What the inflow traces (A_x + B_x eta at xi = -sx, A_y + B_y xi at eta = -sy) of the
// upwind neighbours contribute to the right-hand side of the local system.
template <typename T>
__device__ __forceinline__ void std_inflow(T ax, T ay, T sx, T sy, const T* xin, const T* ydn, T b[4]) {
  const T third = T(1) / T(3);
  b[0] = ax * xin[0] + ay * ydn[0];
  b[1] = -ax * sx * xin[0] + ay * third * ydn[1];
  b[2] = ax * third * xin[1] - ay * sy * ydn[0];
  b[3] = -ax * sx * third * xin[1] - ay * sy * third * ydn[1];
}

// Standard Q^1 sweep: the 4 x 4 local block (sigma_t M + streaming + outflow faces)
// of eq-Ljk with basis 1, xi, eta, xi*eta, right-hand side src (4 moments) plus the
// inflow traces from the left and lower neighbours.  The symmetric part of the block
// is positive definite, so elimination needs no pivoting.  Hands downwind the outflow
// traces; reductions are w c_r (P Psi).
template <typename R>
__device__ __forceinline__ void cell_std(const Dir<R>& d, const R* src, R sigtA, const R* xin,
                                         const R* ydn, R* xo, R* yo, R* o, R* c) {
  const R sx = d.sx, sy = d.sy;
  R m[4][4];
  std_block<R>(sigtA, d.axhy, d.ayhx, d.oxhy, d.oyhx, sx, sy, m);
  R b[4];
  std_inflow<R>(d.axhy, d.ayhx, sx, sy, xin, ydn, b);
#pragma unroll
  for (int k = 0; k < 4; ++k) b[k] += src[k];
  // Gaussian elimination without pivoting
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const R inv = R(1) / m[k][k];
#pragma unroll
    for (int i = k + 1; i < 4; ++i) {
      const R f = m[i][k] * inv;
#pragma unroll
      for (int j = k + 1; j < 4; ++j) m[i][j] -= f * m[k][j];
      b[i] -= f * b[k];
    }
  }
#pragma unroll
  for (int k = 3; k >= 0; --k) {
    R acc = b[k];
#pragma unroll
    for (int j = k + 1; j < 4; ++j) acc -= m[k][j] * c[j];
    c[k] = acc / m[k][k];
  }
  xo[0] = c[0] + sx * c[1];
  xo[1] = c[2] + sx * c[3];
  yo[0] = c[0] + sy * c[2];
  yo[1] = c[1] + sy * c[3];
#pragma unroll
  for (int r = 0; r < 4; ++r) o[r] = d.w * c[r];
}

// ---------------------------------------------------------------- staged sources
// FP64 inputs of one cell (sweep-order column c, row jr) of quadrant (sxi, syi).
//   LMDG/RLMDG: x_0 at the cell, 1 and 2 cells upwind in x and in y; the xi slope
//               of x_1 at the cell and its x-upwind neighbour; the eta slope at the cell
//               and its y-upwind neighbour; sigma_t|K|, eps sigma_a|K|, sigma_s/eps|K|, eps q|K|
//   STD:        the 4 moments at the cell, at its x-upwind and y-upwind neighbours,
//               and the same four material values
// Values outside the mesh are zero (zero exterior traces, vacuum inflow).
template <typename R, int S, bool VAR = false>
__device__ __forceinline__ void raw_load(const SweepParams<R>& P, const double* x, const double* qA, int sxi, int syi,
                                         int c, int jr, double* raw) {
  constexpr int NRAW = SrcTraitsV<S, VAR>::NRAW;
#pragma unroll
  for (int k = 0; k < NRAW; ++k) raw[k] = 0.0;
  if (c < 0 || c >= P.nx || jr >= P.ny) return;
  const int nx = P.nx;
  const long long nc = P.ncell;
  const int i = sxi > 0 ? c : nx - 1 - c;
  const int j = syi > 0 ? jr : P.ny - 1 - jr;
  const long long cell = (long long)j * nx + i;
  const long long sxs = sxi, sys = (long long)syi * nx;  // cell - sxs, cell - sys: upwind
  if constexpr (S == LMDG_SCHEME_STD) {
    if (x) {
#pragma unroll
      for (int m = 0; m < 4; ++m) raw[m] = x[m * nc + cell];
      if (c > 0) {
#pragma unroll
        for (int m = 0; m < 4; ++m) raw[4 + m] = x[m * nc + cell - sxs];
      }
      if (jr > 0) {
#pragma unroll
        for (int m = 0; m < 4; ++m) raw[8 + m] = x[m * nc + cell - sys];
      }
    }
    raw[12] = P.sigtA[cell];
    raw[13] = P.absA[cell];
    raw[14] = P.scatA[cell];
    raw[15] = qA ? qA[cell] : 0.0;
    if (P.qS) {
#pragma unroll
      for (int m = 0; m < 3; ++m) raw[16 + m] = P.qS[m * nc + cell];
    }
  } else {
    if (x) {
      raw[0] = x[cell];
      if (c > 0) raw[1] = x[cell - sxs];
      if (c > 1) raw[2] = x[cell - 2 * sxs];
      if (jr > 0) raw[3] = x[cell - sys];
      if (jr > 1) raw[4] = x[cell - 2 * sys];
      raw[5] = x[nc + cell];
      if (c > 0) raw[6] = x[nc + cell - sxs];
      raw[7] = x[2 * nc + cell];
      if (jr > 0) raw[8] = x[2 * nc + cell - sys];
    }
    raw[9] = P.sigtA[cell];
    raw[10] = P.absA[cell];
    raw[11] = P.scatA[cell];
    raw[12] = qA ? qA[cell] : 0.0;
    if constexpr (VAR) {
      // cross sections of the two upwind neighbours along x and along y
      if (c > 0) { raw[13] = P.scatA[cell - sxs]; raw[14] = P.absA[cell - sxs]; }
      if (c > 1) { raw[15] = P.scatA[cell - 2 * sxs]; raw[16] = P.absA[cell - 2 * sxs]; }
      if (jr > 0) { raw[17] = P.scatA[cell - sys]; raw[18] = P.absA[cell - sys]; }
      if (jr > 1) { raw[19] = P.scatA[cell - 2 * sys]; raw[20] = P.absA[cell - 2 * sys]; }
    }
  }
}

// Upwind rule (a_up, a_uu) along one axis of a cell with `pos` upwind cells inside the
// mesh out of `len`; same1: the cell and its upwind neighbour have the same cross
// sections, same2: that neighbour and the next one do.  rflags: bit 0 three-cell
// stencil, bit 1 suppression at cross-section jumps, bit 3 the adjoint sweep (k = 1 in
// the last cell of the line, 1/2 elsewhere).
__device__ __forceinline__ void upwind_rule(int pos, int len, bool same1, bool same2, int rflags, double& a_up,
                                            double& a_uu) {
  const bool three = rflags & 1, suppress = rflags & 2;
  if (rflags & 8) { a_up = (pos == len - 1) ? 1.0 : 0.5; a_uu = 0.0; }
  else if (pos == 0) { a_up = 1.0; a_uu = 0.0; }
  else if (suppress && !same1) { a_up = 0.0; a_uu = 0.0; }
  else if (three && pos >= 2 && !(suppress && !same2)) { a_up = 1.0; a_uu = 0.25; }
  else { a_up = 0.5; a_uu = 0.0; }
}

// Source coefficients of one cell (FP64 arithmetic, stored in the sweep precision).
//
// LMDG/RLMDG, plain form: M_0 x_0 + L_01 Sigma^T x_1 (+ Q~_0); the isotropic slopes
//   of x_1 enter the constant row through the face traces:
//   c0 = (sigma_s/eps)|K| x_0 + eps q|K|, c1 = h_y (a_K - a_left), c2 = h_x (b_K - b_down).
// LMDG/RLMDG, defect form: (L~_00 Sigma_0^T - M_0) x_0 - L_01 Sigma^T x_1, the same
//   operator rearranged (Sigma_0^T copies x_0 to every direction; P_0 Sigma_0^T = I):
//     x_0 - P_0 L~_00^{-1}(M_0 x_0 + L_01 Sigma^T x_1) = P_0 L~_00^{-1}(defect source).
//   The sigma_s/eps parts of sigma_t|K| and M_0 cancel exactly, leaving
//   c0 = eps sigma_a|K| x_0, c1, c2 = minus the plain ones, c3 = h_y (T_x(K) - T_x(left)),
//   c4 = h_x (T_y(K) - T_y(down)), with T the outflow trace of x_0 (x_0 itself for
//   LMDG; with the upwind slope k (u - u_up), k = 1 in the inflow cell and 1/2
//   inside, for RLMDG; zero outside the mesh).
// STD, plain: M Phi_K = (sigma_s/eps)|K| diag(1, 1/3, 1/3, 1/9) Phi_K (+ Q).
// STD, defect: (L_l Sigma^T - M) Phi = (eps sigma_a|K| mass + streaming + outflow) Phi_K
//   minus the inflow terms of the upwind cells' outflow traces of Phi, split by the
//   factor (1, Ox, Oy, |Ox|, |Oy|) each term carries.
// Within a quadrant Ox = sx |Ox| and Oy = sy |Oy|, so the five factors fold into
// three stored coefficients per moment: src = a + |Ox| b + |Oy| c.
template <typename R, int S, bool VAR = false>
__device__ __forceinline__ void raw_coef(const double* raw, int c, int jr, int sxi, int syi, double hx,
                                         double hy, bool defect, R* coef, int cstride, int rflags = 0, int nx = 0,
                                         int ny = 0) {
  if constexpr (S == LMDG_SCHEME_STD) {
    const double* p = raw;       // moments at the cell
    const double* u = raw + 4;   // x-upwind neighbour
    const double* dn = raw + 8;  // y-upwind neighbour
    const double sigtA = raw[12], absA = raw[13], scatA = raw[14], qA = raw[15];
    const double t3 = 1.0 / 3.0, t9 = 1.0 / 9.0;
    double cf[4][5];
    for (int m = 0; m < 4; ++m)
      for (int k = 0; k < 5; ++k) cf[m][k] = 0.0;
    const double mass[4] = {1.0, t3, t3, t9};
    const double sx = sxi, sy = syi;
    if (!defect) {
      for (int m = 0; m < 4; ++m) cf[m][0] = scatA * mass[m] * p[m];
    } else {
      for (int m = 0; m < 4; ++m) cf[m][0] = absA * mass[m] * p[m];
      // streaming -int u Omega.grad v
      cf[1][1] = -2.0 * hy * p[0];
      cf[3][1] = -2.0 * t3 * hy * p[2];
      cf[2][2] = -2.0 * hx * p[0];
      cf[3][2] = -2.0 * t3 * hx * p[1];
      // outflow faces minus inflow traces of the upwind cells
      const double Ax = u[0] + sx * u[1], Bx = u[2] + sx * u[3];
      const double Ay = dn[0] + sy * dn[2], By = dn[1] + sy * dn[3];
      cf[0][3] = hy * (p[0] + sx * p[1] - Ax);
      cf[1][3] = hy * (sx * p[0] + p[1] + sx * Ax);
      cf[2][3] = hy * (t3 * p[2] + sx * t3 * p[3] - t3 * Bx);
      cf[3][3] = hy * (sx * t3 * p[2] + t3 * p[3] + sx * t3 * Bx);
      cf[0][4] = hx * (p[0] + sy * p[2] - Ay);
      cf[1][4] = hx * (t3 * p[1] + sy * t3 * p[3] - t3 * By);
      cf[2][4] = hx * (sy * p[0] + p[2] + sy * Ay);
      cf[3][4] = hx * (sy * t3 * p[1] + t3 * p[3] + sy * t3 * By);
    }
    cf[0][0] += qA;
    for (int m = 1; m < 4; ++m) cf[m][0] += raw[15 + m];  // source slope moments
    coef[0] = (R)sigtA;
    for (int m = 0; m < 4; ++m) {
      // within a quadrant Ox = sx |Ox| and Oy = sy |Oy|
      coef[(1 + 3 * m) * cstride] = (R)cf[m][0];
      coef[(2 + 3 * m) * cstride] = (R)(sx * cf[m][1] + cf[m][3]);
      coef[(3 + 3 * m) * cstride] = (R)(sy * cf[m][2] + cf[m][4]);
    }
  } else {
    const double x0 = raw[0], u1 = raw[1], u2 = raw[2], d1 = raw[3], d2 = raw[4];
    const double da = hy * (raw[5] - raw[6]);  // h_y (a_K - a_left)
    const double db = hx * (raw[7] - raw[8]);  // h_x (b_K - b_down)
    const double sigtA = raw[9], absA = raw[10], scatA = raw[11], qA = raw[12];
    double c0, c1, c2, c3 = 0.0, c4 = 0.0;
    if (!defect) {
      c0 = scatA * x0 + qA;
      c1 = da;
      c2 = db;
    } else {
      double tx = x0, txu = u1, ty = x0, tyd = d1;
      if (S == LMDG_SCHEME_RLMDG) {
        tx = x0 + (c == 0 ? 1.0 : 0.5) * (x0 - u1);
        ty = x0 + (jr == 0 ? 1.0 : 0.5) * (x0 - d1);
        txu = c > 0 ? u1 + (c == 1 ? 1.0 : 0.5) * (u1 - u2) : 0.0;
        tyd = jr > 0 ? d1 + (jr == 1 ? 1.0 : 0.5) * (d1 - d2) : 0.0;
      }
      c0 = absA * x0 + qA;
      c1 = -da;
      c2 = -db;
      c3 = hy * (tx - txu);
      c4 = hx * (ty - tyd);
    }
    coef[0] = (R)sigtA;
    coef[1 * cstride] = (R)c0;
    coef[2 * cstride] = (R)(sxi * c1 + c3);  // |Ox| factor (Ox = sx |Ox| in the quadrant)
    coef[3 * cstride] = (R)(syi * c2 + c4);  // |Oy| factor
    if (S == LMDG_SCHEME_RLMDG) coef[4 * cstride] = (R)(absA * (1.0 / 3.0));
    if constexpr (VAR) {
      // upwind rules along x and y (no y rule on slab handles, rflags bit 2 clear)
      // cross sections (sigma_s/eps |K|, eps sigma_a |K|): cell raw[11], raw[10]; x-upwind
      // raw[13], raw[14] and the next raw[15], raw[16]; y likewise at raw[17..20]
      const bool same1x = raw[11] == raw[13] && raw[10] == raw[14];
      const bool same2x = raw[13] == raw[15] && raw[14] == raw[16];
      const bool same1y = raw[11] == raw[17] && raw[10] == raw[18];
      const bool same2y = raw[17] == raw[19] && raw[18] == raw[20];
      double axu, axuu, ayu, ayuu;
      upwind_rule(c, nx, same1x, same2x, rflags, axu, axuu);
      upwind_rule(jr, ny, same1y, same2y, rflags, ayu, ayuu);
      if (!(rflags & 4)) ayu = ayuu = 0.0;
      coef[5 * cstride] = (R)axu;
      coef[6 * cstride] = (R)axuu;
      coef[7 * cstride] = (R)ayu;
      coef[8 * cstride] = (R)ayuu;
    }
  }
}

// MAXW bounds the waves per workgroup so that small direction sets get more registers.
// DIRECT: each wave writes its own quadrature sums straight to its slice of the
// partials, [quadrant][wave][NOUT][n_cells], summed over the slices by the combine; this
// takes the cross-wave reduction out of the chunk loop, which pays when few work items
// run (one source on a small mesh).  Otherwise the waves' sums are first added through
// LDS and the partials have one slice per quadrant.
// DATA: source sweeps with prescribed inflow or direction-dependent sources.  The
// inflow datum of eq-main enters as the trace of a ghost cell upwind of the inflow
// face, so that each local solve and reduction takes it exactly where it takes an
// upwind neighbour's trace: per direction and inflow face, alpha supplies (a0, a1, m),
// the face average and the linear Legendre coefficient along the face of alpha, and
// its value at the face midpoint, which is what an upwind cell hands over (STD: the
// trace a0 + a1 t; LMDG: its average; RLMDG: trace average, its linear coefficient
// and the upwind value that the reconstruction of Sec. 3.3.1 takes in the inflow
// cell).  Per-direction source moments are added to the staged isotropic source.
// VAR (RLMDG): the reconstruction variants, with a per-cell upwind rule staged beside
// the source coefficients (cell_rlmdg_var); used with the plain form of the source.
// P1R: also the P_1 R rows of RLMDG (read by the recovery and by lmdg_sweep's output;
// operator applications and right-hand sides skip them).
template <typename R, int S, int MAXW, bool DIRECT, bool DATA = false, bool VAR = false, bool P1R = true>
__global__ void __launch_bounds__(64 * MAXW) sweep2d_kernel(SweepParams<R> P) {
  static_assert(!VAR || S == LMDG_SCHEME_RLMDG, "reconstruction variants are RLMDG sweeps");
  constexpr int NOUT_ALL = SchemeTraits<S>::NOUT;   // partial rows per cell (layout stride)
  constexpr int NOUT = (S == LMDG_SCHEME_RLMDG && !P1R) ? 4 : NOUT_ALL;  // rows produced
  constexpr int NOUTP = (NOUT + 3) & ~3;  // rows of red, padded to whole lane groups
  constexpr int NF = SrcTraitsV<S, VAR>::NF;
  constexpr int NS = SrcTraits<S>::NS;
  constexpr int NC = SrcTraitsV<S, VAR>::NC;
  constexpr int NRAW = SrcTraitsV<S, VAR>::NRAW;
  // staged cells per thread: the 9-wave variant has threads for a whole chunk
  constexpr int MAXC = MAXW > 4 ? 1 : SrcTraits<S>::MAXC;
  // strip-below traces of a chunk per thread: cw NF dslots of them over 64 W threads
  // (dslots = 4 W, chunks of at most 16 columns)
  constexpr int MAXE = NF;
  constexpr bool LM = S != LMDG_SCHEME_STD;
  constexpr bool YRUN = sizeof(R) == 4;  // strip-top traces staged in LDS and stored per chunk
  extern __shared__ unsigned char smem_raw[];
  __shared__ int s_item;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int W = blockDim.x >> 6;
  const int r = lane & 15;
  const int slot = wv * 4 + (lane >> 4);
  const long long nc = P.ncell;
  const int nx = P.nx, ny = P.ny;
  const int lcw = P.lcw;
  const int cw = 1 << lcw;
  const int ncells = kRows << lcw;  // cells staged per chunk
  // LDS: red [cw][W][NOUTP][16] (not with DIRECT) | coef [2][NC][cw][16] | eds [cw][NF][dslots]
  //      | FP32: ybuf [cw][NF][dslots] (row 15's traces of the chunk, written out after its steps)
  // (coefficients structure-of-arrays: the 16 rows of one value are contiguous, so
  // 64-bit reads by the 16 rows of a wave hit distinct banks)
  R* red = reinterpret_cast<R*>(smem_raw);
  // one column's block of red holds W x NOUTP x 16 values plus one pad, so that the
  // reduction's reads of consecutive columns fall in different banks
  const int red_tt = W * NOUTP * kRows + 1;
  R* coef = red + (DIRECT ? 0 : (size_t)cw * red_tt);
  R* eds = coef + (size_t)2 * ncells * NC;
  R* ybuf = eds + (size_t)cw * NF * P.dslots;
  const int nsl = DIRECT ? 4 * W : 4;  // slices of the partials per right-hand side

  for (;;) {
    if (tid == 0) s_item = (int)(atomicAdd(P.ticket, 1u) - P.ticket_base);
    __syncthreads();
    const int item = s_item;
    if (item >= P.n_items) break;
    // item = (strip * n_rhs + rhs) * nq + selected quadrant: every item comes after the
    // one it waits for (same quadrant and right-hand side, strip below)
    const int q = P.qsel[item % P.nq];
    const int s = (item / P.nq) / P.n_rhs;
    const int rh = (item / P.nq) - s * P.n_rhs;
    const double* xr = P.x ? P.x + (long long)rh * 4 * nc : nullptr;
    const double* qAr = P.qA ? P.qA + (long long)rh * nc : nullptr;
    R* const partr = P.part + (long long)rh * nsl * NOUT_ALL * nc;
    R* const edger = P.edge + rh * P.edge_rstride;
    unsigned long long* const progr = P.prog + (long long)rh * 4 * P.nstrips;
    double* const psir = P.psi ? P.psi + rh * P.psi_rstride : nullptr;
    const int sxi = (q & 1) ? -1 : 1;
    const int syi = (q & 2) ? -1 : 1;

    Dir<R> d;
    {
      const double* e = P.dirs + ((long long)q * P.dslots + slot) * kDirStride;
      d.ox = e[0];
      d.oy = e[1];
      d.aox = (R)fabs(d.ox);
      d.aoy = (R)fabs(d.oy);
      d.w = (R)e[2];
      d.idx = (int)e[3];
      d.axhy = (R)(fabs(d.ox) * P.hy);
      d.ayhx = (R)(fabs(d.oy) * P.hx);
      d.oxhy = (R)(d.ox * P.hy);
      d.oyhx = (R)(d.oy * P.hx);
      d.sx = (R)sxi;
      d.sy = (R)syi;
    }
    const int jr = s * kRows + r;  // row in sweep order
    const bool row_ok = jr < ny;
    const int j = syi > 0 ? jr : ny - 1 - jr;
    // slab handles (every Omega_y = 0) reconstruct along x only: a y slope would only
    // feed the decoupled eta rows, whose block scales with eps sigma_a
    const R ky = P.recon_y ? ((jr == 0) ? R(1) : R(0.5)) : R(0);

    // staging of chunk k's cells: thread handles cells e = tid + m * blockDim,
    // e -> (row e / cw, step e % cw) so consecutive threads read consecutive columns
    double raw[MAXC][NRAW];
    auto stage_load = [&](int k) {
#pragma unroll
      for (int m = 0; m < MAXC; ++m) {
        const int e = tid + m * blockDim.x;
        const int rr = e >> lcw, tt = e & (cw - 1);
        const int c = (e < ncells) ? (k << lcw) + tt - rr : -1;
        raw_load<R, S, VAR>(P, xr, qAr, sxi, syi, c, s * kRows + rr, raw[m]);
      }
    };
    auto stage_store = [&](int k, int buf) {
#pragma unroll
      for (int m = 0; m < MAXC; ++m) {
        const int e = tid + m * blockDim.x;
        if (e < ncells) {
          const int rr = e >> lcw, tt = e & (cw - 1);
          raw_coef<R, S, VAR>(raw[m], (k << lcw) + tt - rr, s * kRows + rr, sxi, syi, P.hx, P.hy, P.defect != 0,
                              coef + (size_t)buf * NC * ncells + (tt << 4) + rr, ncells, P.rflags, P.nx, P.ny);
        }
      }
    };

    R xin[NF], yprev[NF], gx[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) { xin[f] = 0; yprev[f] = 0; gx[f] = 0; }
    unsigned long long seen = 0;  // progress word of strip s - 1 last read (thread 0)
    if constexpr (DATA) {
      // ghost trace at the x-inflow face of this lane's row (mesh row j)
      if (P.alpha && row_ok && d.idx >= 0) {
        const double* a = P.alpha + ((long long)d.idx * P.nfaces + j) * 3;
#pragma unroll
        for (int f = 0; f < NF; ++f) gx[f] = f < 3 ? (R)a[f] : R(0);
      }
    }

    stage_load(0);
    stage_store(0, 0);
    for (int k = 0; k < P.nchunks; ++k) {
      const int t0 = k << lcw;
      const int buf = k & 1;
      // wait until strip s - 1 has completed the chunk's columns: thread 0 keeps the
      // progress word it last read and reads it again only while that falls short
      if (s > 0 && tid == 0) {
        const int need = min(nx, t0 + cw);
        const unsigned long long target = ((P.epoch + P.wait_bias) << 32) | (unsigned long long)need;
        if (seen < target) {
          const unsigned long long* flag = progr + (long long)q * P.nstrips + (s - 1);
          long long spins = 0;
          while ((seen = load_agent(flag)) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > P.spin_limit) { atomicOr(P.err, 1); break; }
          }
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
      }
      __syncthreads();
      // traces of the strip below for the columns of this chunk (zero for the first strip):
      // all of a thread's loads issued at once (addresses clamped into the buffer, values
      // outside the mesh replaced by zero afterwards), then written to LDS, so that the
      // chunk waits for one memory latency
      {
        const int ne = (cw * NF) * P.dslots;
        const int ne_in = s > 0 ? max(0, min(cw, nx - t0)) * NF * P.dslots : 0;  // columns inside the mesh
        const R* src = edger + (((long long)q * P.nstrips + max(s - 1, 0)) * nx + (t0 < nx ? t0 : 0)) * NF * P.dslots;
        R ev[MAXE];
#pragma unroll
        for (int kk = 0; kk < MAXE; ++kk) {
          const int e = tid + kk * (int)blockDim.x;
          const R v = load_agent(src + (e < ne_in ? e : 0));
          ev[kk] = e < ne_in ? v : R(0);
        }
#pragma unroll
        for (int kk = 0; kk < MAXE; ++kk) {
          const int e = tid + kk * (int)blockDim.x;
          if (e >= ne) continue;
          const int c = t0 + e / (NF * P.dslots);
          R v = ev[kk];
          if constexpr (DATA) {
            // ghost traces below the y-inflow faces of the first strip
            if (s == 0 && P.alpha && c < nx) {
              const int sl = e % P.dslots, f = (e / P.dslots) % NF;
              const int l = (int)P.dirs[((long long)q * P.dslots + sl) * kDirStride + 3];
              const int i = sxi > 0 ? c : nx - 1 - c;
              if (l >= 0 && f < 3) v = (R)P.alpha[((long long)l * P.nfaces + ny + i) * 3 + f];
            }
          }
          eds[e] = v;
        }
      }
      if (k + 1 < P.nchunks) stage_load(k + 1);  // overlaps the step loop below
      lds_barrier();  // staged traces and coefficients visible; the prefetch stays in flight

      const R* cbuf = coef + (size_t)buf * NC * ncells;
      // Steps run in fully unrolled groups of U: the source, sigma_t, reciprocal of the
      // denominator and strip-below trace of all U steps (none depends on upwind
      // values) are formed first as independent chains, then the U dependent steps
      // follow; the body has no branches except the stores after each group, so one
      // wave can overlap the latencies itself.
      constexpr int U = step_group<R>();
      for (int tg = 0; tg < cw; tg += U) {
        R src_g[U][NS], sig_g[U], inv_g[U], edn_g[U][NF], ru_g[U][VAR ? 4 : 1];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int tt = tg + u;
          const R* cf = cbuf + (tt << 4) + r;
          sig_g[u] = cf[0];
#pragma unroll
          for (int m = 0; m < NS; ++m) {
            const R* a = cf + (size_t)(1 + 3 * m) * ncells;
            src_g[u][m] = a[0] + d.aox * a[ncells] + d.aoy * a[2 * ncells];
          }
          if constexpr (DATA) {
            const int c = t0 + tt - r;
            if (P.qdir && row_ok && d.idx >= 0 && c >= 0 && c < nx) {
              const long long cell = (long long)j * nx + (sxi > 0 ? c : nx - 1 - c);
#pragma unroll
              for (int m = 0; m < NS; ++m) src_g[u][m] += (R)P.qdir[((long long)d.idx * P.qdir_nm + m) * nc + cell];
            }
          }
          if constexpr (S == LMDG_SCHEME_LMDG) {
            inv_g[u] = recip(sig_g[u] + d.axhy + d.ayhx);
          } else if constexpr (VAR) {
#pragma unroll
            for (int e = 0; e < 4; ++e) ru_g[u][e] = cf[(5 + e) * ncells];
            inv_g[u] = recip(sig_g[u] + d.axhy * (R(1) + ru_g[u][0] - ru_g[u][1]) +
                             d.ayhx * (R(1) + ru_g[u][2] - ru_g[u][3]));
          } else if constexpr (S == LMDG_SCHEME_RLMDG) {
            const R kx = (t0 + tt - r == 0) ? R(1) : R(0.5);
            inv_g[u] = recip(sig_g[u] + d.axhy * (R(1) + kx) + d.ayhx * (R(1) + ky));
          } else {
            inv_g[u] = R(0);
          }
#pragma unroll
          for (int f = 0; f < NF; ++f) edn_g[u][f] = eds[((tt * NF) + f) * P.dslots + slot];
        }
        R yo_g[U][NF], psi_g[U][4], ov_g[U][NOUTP / 4];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int tt = tg + u;
          const int c = t0 + tt - r;
          const bool act = row_ok && c >= 0 && c < nx;
          const R inv = inv_g[u];
          R ydn[NF];
#pragma unroll
          for (int f = 0; f < NF; ++f) {
            const R v = shr1(yprev[f]);
            ydn[f] = (r == 0) ? edn_g[u][f] : v;
            xin[f] = (c == 0) ? gx[f] : xin[f];
          }
          R o[NOUT_ALL], xo[NF], yo[NF];
          if constexpr (S == LMDG_SCHEME_STD) {
            cell_std<R>(d, src_g[u], sig_g[u], xin, ydn, xo, yo, o, psi_g[u]);
          } else if constexpr (S == LMDG_SCHEME_LMDG) {
            cell_lmdg<R>(d, src_g[u][0], inv, xin, ydn, xo, yo, o, psi_g[u][0]);
          } else if constexpr (VAR) {
            cell_rlmdg_var<R>(d, src_g[u][0], cbuf[((tt << 4) + r) + 4 * ncells], inv, ru_g[u], xin, ydn, xo, yo, o,
                              psi_g[u][0], (P.rflags & 8) != 0);
          } else {
            const R kx = (c == 0) ? R(1) : R(0.5);
            cell_rlmdg<R>(d, src_g[u][0], cbuf[((tt << 4) + r) + 4 * ncells], inv, kx, ky, xin, ydn, xo, yo, o,
                          psi_g[u][0]);
          }
#pragma unroll
          for (int f = 0; f < NF; ++f) {
            xin[f] = xo[f];
            yprev[f] = yo[f];
            yo_g[u][f] = yo[f];
          }
          // sums over the four direction slots of the wave, four rows at a time: lane
          // group g receives row m0 + g (no branch, so the steps of a group stay one
          // scheduling region)
          R om[NOUTP];
#pragma unroll
          for (int m = 0; m < NOUTP; ++m) om[m] = (m < NOUT && act) ? o[m < NOUT ? m : 0] : R(0);
#pragma unroll
          for (int m0 = 0; m0 < NOUTP; m0 += 4) {
            const R v = quad_sum4(om[m0], om[m0 + 1], om[m0 + 2], om[m0 + 3]);
            if constexpr (DIRECT)
              ov_g[u][m0 >> 2] = v;
            else
              red[tt * red_tt + (wv * NOUTP + m0 + (lane >> 4)) * kRows + r] = v;
          }
        }
        if constexpr (DIRECT) {
          // this wave's sums of the group's cells: lane group g writes rows g, g + 4, ...
          const int g4 = lane >> 4;
          R* const pw = partr + (long long)(q * W + wv) * NOUT_ALL * nc;
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int c = t0 + tg + u - r;
            if (row_ok && c >= 0 && c < nx) {
              const int i = sxi > 0 ? c : nx - 1 - c;
              const long long cell = (long long)j * nx + i;
#pragma unroll
              for (int m0 = 0; m0 < NOUTP; m0 += 4)
                if (m0 + g4 < NOUT) pw[(long long)(m0 + g4) * nc + cell] = ov_g[u][m0 >> 2];
            }
          }
        }
        if (r == kRows - 1 && s + 1 < P.nstrips) {
          if constexpr (YRUN) {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
              for (int f = 0; f < NF; ++f) ybuf[((tg + u) * NF + f) * P.dslots + slot] = yo_g[u][f];
          } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const int c = t0 + tg + u - r;
              if (row_ok && c >= 0 && c < nx) {
                R* e = edger + ((((long long)q * P.nstrips + s) * nx + c) * NF) * P.dslots + slot;
#pragma unroll
                for (int f = 0; f < NF; ++f) store_agent(e + (long long)f * P.dslots, yo_g[u][f]);
              }
            }
          }
        }
        if (psir && d.idx >= 0) {
          const int pdir = P.psi_by_slot ? slot : d.idx;
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int c = t0 + tg + u - r;
            if (row_ok && c >= 0 && c < nx) {
              const int i = sxi > 0 ? c : nx - 1 - c;
              const long long cell = (long long)j * nx + i;
              if constexpr (LM) {
                psir[(long long)pdir * nc + cell] = (double)psi_g[u][0];
              } else {
#pragma unroll
                for (int m = 0; m < 4; ++m) psir[((long long)pdir * 4 + m) * nc + cell] = (double)psi_g[u][m];
              }
            }
          }
        }
      }
      // FP32: the chunk's strip-top traces, columns t0 - 15 .. t0 + cw - 16 inside the mesh,
      // as one contiguous run (stored from row 15 per step, each wave's direction slots
      // fall into short pieces of a column's run; in FP64 the extra barrier and LDS cost
      // more than the pieces)
      if (YRUN && s + 1 < P.nstrips) {
        lds_barrier();
        const int nds = NF * P.dslots;
        const int e_lo = max(0, kRows - 1 - t0) * nds, e_hi = min(cw, nx - t0 + kRows - 1) * nds;
        const long long base = (((long long)q * P.nstrips + s) * nx + (t0 - (kRows - 1))) * nds;
        for (int e = e_lo + tid; e < e_hi; e += blockDim.x) store_agent(edger + (base + e), ybuf[e]);
      }
      // publish this chunk's strip-top traces before the staging and reduction below,
      // which the strip above does not wait for: every wave waits for its own trace
      // stores to complete before the barrier, then one thread releases and raises the flag
      if (s + 1 < P.nstrips) __builtin_amdgcn_s_waitcnt(kWaitVmem);
      __syncthreads();
      if (s + 1 < P.nstrips && tid == 0) {
        const int done = min(nx, t0 + cw - (kRows - 1));
        if (done > 0) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          store_agent(progr + (long long)q * P.nstrips + s, (P.epoch << 32) | (unsigned long long)done);
        }
      }
      if (k + 1 < P.nchunks) stage_store(k + 1, buf ^ 1);
      // sums over waves, written with consecutive threads on consecutive columns
      const int nred = DIRECT ? 0 : (NOUT * kRows) << lcw;
      for (int e = tid; e < nred; e += blockDim.x) {
        const int tt = e & (cw - 1);
        const int m = (e >> lcw) % NOUT;
        const int rr = (e >> lcw) / NOUT;
        const int c = t0 + tt - rr;
        const int jr2 = s * kRows + rr;
        if (jr2 < ny && c >= 0 && c < nx) {
          R acc = 0;
#pragma unroll
          for (int w2 = 0; w2 < MAXW; ++w2)
            if (w2 < W) acc += red[tt * red_tt + (w2 * NOUTP + m) * kRows + rr];
          const int i = sxi > 0 ? c : nx - 1 - c;
          const int jj = syi > 0 ? jr2 : ny - 1 - jr2;
          partr[((long long)q * NOUT_ALL + m) * nc + (long long)jj * nx + i] = acc;
        }
      }
    }
    __syncthreads();
  }
}

template <typename R, int S, bool VAR = false>
size_t lds_bytes(int cw, int W, int dslots, bool direct) {
  constexpr int NOUT = SchemeTraits<S>::NOUT;
  constexpr int NF = SrcTraitsV<S, VAR>::NF;
  constexpr int NC = SrcTraitsV<S, VAR>::NC;
  constexpr int NOUTP = (NOUT + 3) & ~3;
  const size_t red = direct ? 0 : (size_t)cw * (W * NOUTP * kRows + 1);  // cross-wave sums
  const size_t edges = (sizeof(R) == 4 ? 2 : 1) * (size_t)cw * NF * dslots;  // eds (and ybuf in FP32)
  return (red + (size_t)2 * cw * kRows * NC + edges) * sizeof(R);
}

// The plain (no inflow data, default reconstruction) instantiations, with or without the
// P_1 R rows of RLMDG.
template <typename R, int S, int MAXW, bool DIRECT>
void launch_plain(const SweepParams<R>& P, int grid, int W, size_t lds, hipStream_t st, bool p1r) {
  if constexpr (S == LMDG_SCHEME_RLMDG) {
    if (!p1r) {
      hipLaunchKernelGGL((sweep2d_kernel<R, S, MAXW, DIRECT, false, false, false>), dim3(grid), dim3(64 * W), lds, st,
                         P);
      return;
    }
  }
  hipLaunchKernelGGL((sweep2d_kernel<R, S, MAXW, DIRECT>), dim3(grid), dim3(64 * W), lds, st, P);
}

template <typename R, int S>
int launch_typed(lmdg_handle* h, const double* x, bool use_q, double* psi, hipStream_t st, bool defect, int qmask,
                 bool psi_by_slot, bool p1r) {
  SweepParams<R> P;
  P.nx = (int)h->n[0];
  P.ny = (int)h->n[1];
  P.nstrips = h->nstrips;
  P.dslots = h->dslots;
  const int W = h->waves;
  // chunk length: at most MAXC staged cells per thread and kLdsBudget bytes of LDS
  // (one workgroup per compute unit; gfx950 gives a workgroup up to 160 KB)
  constexpr size_t kLdsBudget = 144 * 1024;
  int cw = 16;
  const int maxc = W > 4 ? 1 : SrcTraits<S>::MAXC;
  // inflow data and direction-dependent sources belong to the handle's own source
  // (not to the detector source of an adjoint solve)
  const bool data = use_q && !h->src0 && (h->d_alpha || h->d_qdir);
  // reconstruction variants (RLMDG): their own kernel, always with the plain source
  constexpr bool kRlm = S == LMDG_SCHEME_RLMDG;
  const bool adj = kRlm && h->adj_rlm;  // adjoint sweep of the reconstructed scheme
  const bool var = kRlm && (h->recon_flags != 0 || adj);
  const bool direct = !data && !var && part_slices(h, S, sizeof(R) == 8 ? LMDG_PREC_FP64 : LMDG_PREC_FP32) > 4;
  h->last_nsl = direct ? 4 * W : 4;  // slices of the partials the combine adds
  auto lds_of = [&](int c) {
    return var ? lds_bytes<R, S, kRlm>(c, W, h->dslots, direct) : lds_bytes<R, S>(c, W, h->dslots, direct);
  };
  while (cw > step_group<R>() && (kRows * cw > maxc * 64 * W || lds_of(cw) > kLdsBudget)) cw >>= 1;
  P.cw = cw;
  P.lcw = 0;
  while ((1 << P.lcw) < cw) ++P.lcw;
  P.nchunks = (P.nx + kRows - 1 + cw - 1) / cw;
  P.n_rhs = h->n_rhs;
  P.nq = 0;
  for (int q = 0; q < 4; ++q)
    if (qmask & (1 << q)) P.qsel[P.nq++] = q;
  for (int q = P.nq; q < 4; ++q) P.qsel[q] = 0;
  P.psi_by_slot = psi_by_slot ? 1 : 0;
  P.n_items = P.nq * h->nstrips * h->n_rhs;
  P.hx = h->h[0];
  P.hy = h->h[1];
  P.ncell = h->ncell;
  P.dirs = h->d_dirs;
  P.x = x;
  P.sigtA = h->d_sigtA;
  P.scatA = h->d_scatA;
  P.qA = use_q ? (h->src0 ? h->src0 : h->d_qA) : nullptr;
  P.qS = (use_q && S == LMDG_SCHEME_STD) ? (h->src0 ? h->src1 : h->d_qS) : nullptr;
  P.alpha = (data && !adj) ? h->d_alpha : nullptr;
  P.qdir = adj ? h->d_adjsrc : (data ? h->d_qdir : nullptr);
  P.qdir_nm = adj ? 1 : 4;
  P.nfaces = (int)(h->n[0] + h->n[1]);
  P.recon_y = h->slab ? 0 : 1;
  P.rflags = (adj ? 8 : h->recon_flags) | (h->slab ? 0 : 4);
  P.absA = h->d_absA;
  P.defect = (defect && !var) ? 1 : 0;
  P.part = reinterpret_cast<R*>(h->ws.part);
  P.edge = reinterpret_cast<R*>(h->ws.edge);
  P.psi = psi;
  P.psi_rstride = (long long)h->ndir * (S == LMDG_SCHEME_STD ? 4 : 1) * h->ncell;
  P.edge_rstride = (long long)4 * h->nstrips * P.nx * (SchemeTraits<S>::NF + (var ? 1 : 0)) * h->dslots;
  P.prog = h->ws.prog;
  P.ticket = h->ws.ticket;
  P.err = h->ws.err;
  P.epoch = h->epoch;
  P.ticket_base = h->ticket_base;
  P.spin_limit = h->spin_limit;
  P.wait_bias = h->wait_bias;
  const int grid = std::min(P.n_items, 4 * h->n_cu);
  const size_t lds = lds_of(cw);
  hipEvent_t ev_end = nullptr;
  if (h->profiling) {
    if (h->ev_used + 2 > h->ev_pool.size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        return set_error(h, LMDG_HIP_ERROR, "hipEventCreate");
      h->ev_pool.push_back(a);
      h->ev_pool.push_back(b);
    }
    hipEventRecord(h->ev_pool[h->ev_used], st);
    ev_end = h->ev_pool[h->ev_used + 1];
    h->ev_used += 2;
  }
  if constexpr (kRlm) {
    if (var) {
      if (W <= 4)
        hipLaunchKernelGGL((sweep2d_kernel<R, S, 4, false, true, true>), dim3(grid), dim3(64 * W), lds, st, P);
      else
        hipLaunchKernelGGL((sweep2d_kernel<R, S, kMaxWaves, false, true, true>), dim3(grid), dim3(64 * W), lds, st,
                           P);
    }
  }
  if (var) {
  } else if (data) {
    if (W <= 4)
      hipLaunchKernelGGL((sweep2d_kernel<R, S, 4, false, true>), dim3(grid), dim3(64 * W), lds, st, P);
    else
      hipLaunchKernelGGL((sweep2d_kernel<R, S, kMaxWaves, false, true>), dim3(grid), dim3(64 * W), lds, st, P);
  } else if constexpr (sizeof(R) == 8) {
    if (direct && W <= 4) {
      launch_plain<R, S, 4, true>(P, grid, W, lds, st, p1r);
    } else if (direct) {
      launch_plain<R, S, kMaxWaves, true>(P, grid, W, lds, st, p1r);
    } else if (W <= 4) {
      launch_plain<R, S, 4, false>(P, grid, W, lds, st, p1r);
    } else {
      launch_plain<R, S, kMaxWaves, false>(P, grid, W, lds, st, p1r);
    }
  } else {
    if (W <= 4)
      launch_plain<R, S, 4, false>(P, grid, W, lds, st, p1r);
    else
      launch_plain<R, S, kMaxWaves, false>(P, grid, W, lds, st, p1r);
  }
  if (ev_end) hipEventRecord(ev_end, st);
  h->epoch += 1;
  h->ticket_base += (unsigned)(P.n_items + grid);
  return check_hip(h, hipGetLastError(), "sweep launch");
}

}  // namespace

int launch_sweep(lmdg_handle* h, int scheme, int prec, const double* x, bool use_q, double* psi,
                 hipStream_t st, bool defect, int qmask, bool psi_by_slot, bool p1r) {
  if (h->dim == 3) {
    if (qmask != 0xF || psi_by_slot) return set_error(h, LMDG_UNSUPPORTED, "quadrant-restricted 3D sweep");
    return launch_sweep3d(h, scheme, prec, x, use_q, psi, st, defect, p1r);
  }
  if ((qmask & 0xF) == 0) return set_error(h, LMDG_INVALID_ARG, "empty quadrant mask");
  if (prec == LMDG_PREC_FP64) {
    switch (scheme) {
      case LMDG_SCHEME_STD:
        return launch_typed<double, LMDG_SCHEME_STD>(h, x, use_q, psi, st, defect, qmask, psi_by_slot, true);
      case LMDG_SCHEME_LMDG:
        return launch_typed<double, LMDG_SCHEME_LMDG>(h, x, use_q, psi, st, defect, qmask, psi_by_slot, true);
      default:
        return launch_typed<double, LMDG_SCHEME_RLMDG>(h, x, use_q, psi, st, defect, qmask, psi_by_slot, p1r);
    }
  }
  switch (scheme) {
    case LMDG_SCHEME_STD:
      return launch_typed<float, LMDG_SCHEME_STD>(h, x, use_q, psi, st, defect, qmask, psi_by_slot, true);
    case LMDG_SCHEME_LMDG:
      return launch_typed<float, LMDG_SCHEME_LMDG>(h, x, use_q, psi, st, defect, qmask, psi_by_slot, true);
    default:
      return launch_typed<float, LMDG_SCHEME_RLMDG>(h, x, use_q, psi, st, defect, qmask, psi_by_slot, p1r);
  }
}

}  // namespace lmdg
