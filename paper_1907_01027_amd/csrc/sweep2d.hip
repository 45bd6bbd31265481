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
//   reductions = per-cell sums over directions: over the 4 slots of a wave with two
//                cross-lane swaps, over waves through LDS, written once per cell and
//                quadrant; a combine kernel adds the quadrants.
// Strips publish "columns finished in my top row" every CW steps with an agent-scope
// release; consumers acquire before reading.  Progress words carry the launch epoch
// in the high half so they never need clearing.  Every wait is bounded: a stuck wait
// sets an error flag and the kernel still finishes.
#include "internal.h"

namespace lmdg {
namespace {

__device__ __forceinline__ float shr1(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, false));
}
__device__ __forceinline__ double shr1(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, 0x111, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, 0x111, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum of the four lanes r, r+16, r+32, r+48 (same row, four direction slots),
// returned to all four; the pairing order is fixed, so results are reproducible.
__device__ __forceinline__ float quad_sum(float v) {
  unsigned u = __float_as_uint(v);
  auto a = __builtin_amdgcn_permlane16_swap(u, u, false, false);
  float s = __uint_as_float(a[0]) + __uint_as_float(a[1]);
  unsigned us = __float_as_uint(s);
  auto b = __builtin_amdgcn_permlane32_swap(us, us, false, false);
  return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}
__device__ __forceinline__ double quad_sum(double v) {
  unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
  auto al = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  auto ah = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  double s = __hiloint2double((int)ah[0], (int)al[0]) + __hiloint2double((int)ah[1], (int)al[1]);
  lo = (unsigned)__double2loint(s);
  hi = (unsigned)__double2hiint(s);
  auto bl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  auto bh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double((int)bh[0], (int)bl[0]) + __hiloint2double((int)bh[1], (int)bl[1]);
}

template <typename T>
__device__ __forceinline__ T load_agent(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void store_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr long long kSpinLimit = 1ll << 25;

// Per-lane direction constants.
template <typename R>
struct Dir {
  double ox, oy;        // Omega components
  R w;                  // quadrature weight (0 for padding slots)
  R axhy, ayhx;         // |Omega_x| h_y, |Omega_y| h_x  (face measures times |Omega.nu|)
  R oxhy, oyhx;         // Omega_x h_y, Omega_y h_x
  R sx, sy;             // signs of Omega_x, Omega_y
  int idx;              // caller's direction index, -1 for padding
};

// ---------------------------------------------------------------- local solves
// Low-memory sweep (L_00 of Sec. 3.2): one unknown per cell and direction.
// Row "test with the cell constant" of eq-Ljk:
//   sigma_t|K| psi + |Ox| h_y (psi - psi_left) + |Oy| h_x (psi - psi_down) = src.
// Reductions: w psi (P_0), w Ox h_y (psi_left - psi), w Oy h_x (psi_down - psi)
// (rows xi, eta of Sigma L_10; its xi*eta row vanishes).
template <typename R>
__device__ __forceinline__ void cell_lmdg(const Dir<R>& d, R src, R sigtA, const R* xin, const R* ydn,
                                          R* xo, R* yo, R* o, R& psi_out) {
  const R num = src + d.axhy * xin[0] + d.ayhx * ydn[0];
  const R den = sigtA + d.axhy + d.ayhx;
  const R psi = num / den;
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
// (where the upwind value is the vacuum inflow 0).  A face hands downwind its trace
// average T, its linear coefficient along the face, and the cell average.
// Reductions: w psi, the xi / eta / xi*eta rows of w (L_10 + L_11 R) applied to the
// cell function, and w c_xi, w c_eta (for P_1 R).
template <typename R>
__device__ __forceinline__ void cell_rlmdg(const Dir<R>& d, R src, R sigtA, R kx, R ky, const R* xin,
                                           const R* ydn, R* xo, R* yo, R* o, R& psi_out) {
  // xin = (T_x of left cell, its c_eta, its average); ydn = (T_y, c_xi, average) of cell below
  const R third = R(1) / R(3);
  const R num = src + d.axhy * (xin[0] + kx * xin[2]) + d.ayhx * (ydn[0] + ky * ydn[2]);
  const R den = sigtA + d.axhy * (R(1) + kx) + d.ayhx * (R(1) + ky);
  const R psi = num / den;
  const R cxi = d.sx * kx * (psi - xin[2]);
  const R ceta = d.sy * ky * (psi - ydn[2]);
  const R tx = psi + kx * (psi - xin[2]);
  const R ty = psi + ky * (psi - ydn[2]);
  xo[0] = tx; xo[1] = ceta; xo[2] = psi;
  yo[0] = ty; yo[1] = cxi;  yo[2] = psi;
  const R sA3 = sigtA * third;
  o[0] = d.w * psi;
  o[1] = d.w * (d.oxhy * (xin[0] - psi) + (sA3 + d.axhy + d.ayhx * third) * cxi - d.ayhx * third * ydn[1]);
  o[2] = d.w * (d.oyhx * (ydn[0] - psi) + (sA3 + d.ayhx + d.axhy * third) * ceta - d.axhy * third * xin[1]);
  o[3] = d.w * third * (d.oxhy * (xin[1] - ceta) + d.oyhx * (ydn[1] - cxi));
  o[4] = d.w * cxi;
  o[5] = d.w * ceta;
  psi_out = psi;
}

// Standard Q^1 sweep: the 4 x 4 local block (sigma_t M + streaming + outflow faces)
// of eq-Ljk with basis 1, xi, eta, xi*eta, right-hand side src (4 moments) plus the
// inflow traces A + B (along-face coordinate) from the left and lower neighbours.
// The symmetric part of the block is positive definite, so elimination needs no
// pivoting.  Hands downwind the outflow traces; reductions are w c_r (P Psi).
// Local block (coef M + streaming + outflow faces) of the standard sweep; coef is
// sigma_t|K| for the sweep and eps sigma_a |K| for the defect source below.
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

// ---------------------------------------------------------------- FP64 sources
// Right-hand side of the low-memory sweeps for a moment vector x (FP64), with the
// upwind cells at cell - sxs (x) and cell - sys (y); c, jr are sweep-order indices.
//   plain : M_0 x_0 + L_01 Sigma^T x_1
//   defect: (L~_00 Sigma_0^T - M_0) x_0 - L_01 Sigma^T x_1
// The defect form is the same operator rearranged (Sigma_0^T copies x_0 to every
// direction, P_0 Sigma_0^T = I since the weights sum to one):
//   x_0 - P_0 L~_00^{-1}(M_0 x_0 + L_01 Sigma^T x_1) = P_0 L~_00^{-1}(defect source);
// the sigma_s/eps parts of sigma_t|K| and M_0 cancel exactly, leaving eps sigma_a |K|
// and upwind face differences of x_0, so nothing large cancels after the sweep.
// L~_00 applied to an isotropic field u: sigma_t|K| u_K + |Ox| h_y (T_x(K) - T_x(up))
// + |Oy| h_x (T_y(K) - T_y(down)), T = outflow trace (u itself for LMDG; with the
// upwind slope k (u - u_up), k = 1 in the inflow cell and 1/2 inside, for RLMDG;
// zero for cells outside the mesh).
template <bool REC>
__device__ __forceinline__ double lm_source(const double* x, long long nc, long long cell, long long sxs,
                                            long long sys, int c, int jr, double scatA, double absA, double ox,
                                            double oy, double hx, double hy, bool defect) {
  const double a = x[nc + cell], b = x[2 * nc + cell];
  const double al = c > 0 ? x[nc + cell - sxs] : 0.0;
  const double bd = jr > 0 ? x[2 * nc + cell - sys] : 0.0;
  const double l01 = ox * hy * (a - al) + oy * hx * (b - bd);
  const double x0 = x[cell];
  if (!defect) return scatA * x0 + l01;
  const double u1 = c > 0 ? x[cell - sxs] : 0.0;
  const double d1 = jr > 0 ? x[cell - sys] : 0.0;
  double tx = x0, txu = u1, ty = x0, tyd = d1;
  if (REC) {
    const double u2 = c > 1 ? x[cell - 2 * sxs] : 0.0;
    const double d2 = jr > 1 ? x[cell - 2 * sys] : 0.0;
    tx = x0 + (c == 0 ? 1.0 : 0.5) * (x0 - u1);
    ty = x0 + (jr == 0 ? 1.0 : 0.5) * (x0 - d1);
    txu = c > 0 ? u1 + (c == 1 ? 1.0 : 0.5) * (u1 - u2) : 0.0;
    tyd = jr > 0 ? d1 + (jr == 1 ? 1.0 : 0.5) * (d1 - d2) : 0.0;
  }
  return absA * x0 + fabs(ox) * hy * (tx - txu) + fabs(oy) * hx * (ty - tyd) - l01;
}

// Right-hand side of the standard sweep for Phi = x (FP64, 4 moments):
//   plain : M Phi_K = (sigma_s/eps)|K| diag(1, 1/3, 1/3, 1/9) Phi_K
//   defect: (L_l Sigma^T - M) Phi = (eps sigma_a |K| mass + streaming + outflow) Phi_K
//           minus the inflow terms built from the upwind cells' outflow traces of Phi,
// so that Phi - P L^{-1} M Phi = P L^{-1}(defect source) without cancellation.
__device__ __forceinline__ void std_source(const double* x, long long nc, long long cell, long long sxs,
                                           long long sys, int c, int jr, double scatA, double absA, double ox,
                                           double oy, double hx, double hy, bool defect, double out[4]) {
  const double phi[4] = {x[cell], x[nc + cell], x[2 * nc + cell], x[3 * nc + cell]};
  if (!defect) {
    out[0] = scatA * phi[0];
    out[1] = scatA * (1.0 / 3.0) * phi[1];
    out[2] = scatA * (1.0 / 3.0) * phi[2];
    out[3] = scatA * (1.0 / 9.0) * phi[3];
    return;
  }
  const double sx = ox > 0 ? 1.0 : -1.0, sy = oy > 0 ? 1.0 : -1.0;
  const double ax = fabs(ox) * hy, ay = fabs(oy) * hx;
  double m[4][4];
  std_block<double>(absA, ax, ay, ox * hy, oy * hx, sx, sy, m);
#pragma unroll
  for (int r = 0; r < 4; ++r) out[r] = m[r][0] * phi[0] + m[r][1] * phi[1] + m[r][2] * phi[2] + m[r][3] * phi[3];
  double xin[2] = {0.0, 0.0}, ydn[2] = {0.0, 0.0};
  if (c > 0) {
    const long long u = cell - sxs;
    xin[0] = x[u] + sx * x[nc + u];
    xin[1] = x[2 * nc + u] + sx * x[3 * nc + u];
  }
  if (jr > 0) {
    const long long u = cell - sys;
    ydn[0] = x[u] + sy * x[2 * nc + u];
    ydn[1] = x[nc + u] + sy * x[3 * nc + u];
  }
  double b[4];
  std_inflow<double>(ax, ay, sx, sy, xin, ydn, b);
#pragma unroll
  for (int r = 0; r < 4; ++r) out[r] -= b[r];
}

template <typename R, int S>
__global__ void __launch_bounds__(1024) sweep2d_kernel(SweepParams<R> P) {
  constexpr int NOUT = SchemeTraits<S>::NOUT;
  constexpr int NF = SchemeTraits<S>::NF;
  extern __shared__ unsigned char smem_raw[];
  R* red = reinterpret_cast<R*>(smem_raw);  // [cw][W][NOUT][16]
  __shared__ int s_item;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int W = blockDim.x >> 6;
  const int r = lane & 15;
  const int slot = wv * 4 + (lane >> 4);
  const long long nc = P.ncell;
  const int nx = P.nx, ny = P.ny;

  for (;;) {
    if (tid == 0) s_item = (int)(atomicAdd(P.ticket, 1u) - P.ticket_base);
    __syncthreads();
    const int item = s_item;
    if (item >= P.n_items) break;
    const int q = item & 3;
    const int s = item >> 2;
    const int sxi = (q & 1) ? -1 : 1;
    const int syi = (q & 2) ? -1 : 1;

    Dir<R> d;
    {
      const double* e = P.dirs + ((long long)q * P.dslots + slot) * kDirStride;
      d.ox = e[0];
      d.oy = e[1];
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
    const R ky = (jr == 0) ? R(1) : R(0.5);

    R xin[NF], yprev[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) { xin[f] = 0; yprev[f] = 0; }

    for (int k = 0; k < P.nchunks; ++k) {
      const int t0 = k * P.cw;
      if (s > 0 && tid == 0) {
        const int need = min(nx, t0 + P.cw);
        const unsigned long long target = (P.epoch << 32) | (unsigned long long)need;
        const unsigned long long* flag = P.prog + (long long)q * P.nstrips + (s - 1);
        long long spins = 0;
        while (load_agent(flag) < target) {
          __builtin_amdgcn_s_sleep(2);
          if (++spins > kSpinLimit) { atomicOr(P.err, 1); break; }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      __syncthreads();

      for (int tt = 0; tt < P.cw; ++tt) {
        const int c = t0 + tt - r;
        const bool act = row_ok && c >= 0 && c < nx;
        R ydn[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) ydn[f] = shr1(yprev[f]);
        if (r == 0) {
          if (act && s > 0) {
            const R* e = P.edge + ((((long long)q * P.nstrips + (s - 1)) * nx + c) * NF) * P.dslots + slot;
#pragma unroll
            for (int f = 0; f < NF; ++f) ydn[f] = load_agent(e + (long long)f * P.dslots);
          } else {
#pragma unroll
            for (int f = 0; f < NF; ++f) ydn[f] = 0;
          }
        }
        if (c == 0) {
#pragma unroll
          for (int f = 0; f < NF; ++f) xin[f] = 0;
        }
        R o[NOUT], xo[NF], yo[NF];
#pragma unroll
        for (int m = 0; m < NOUT; ++m) o[m] = 0;
#pragma unroll
        for (int f = 0; f < NF; ++f) { xo[f] = xin[f]; yo[f] = 0; }
        if (act) {
          const int i = sxi > 0 ? c : nx - 1 - c;
          const long long cell = (long long)j * nx + i;
          const double sigtA = P.sigtA[cell];
          const long long sxs = sxi, sys = (long long)syi * nx;  // cell - sxs / - sys = upwind
          if constexpr (S == LMDG_SCHEME_STD) {
            R src[4];
            double sd[4] = {0, 0, 0, 0};
            if (P.x)
              std_source(P.x, nc, cell, sxs, sys, c, jr, P.scatA[cell], P.absA[cell], d.ox, d.oy, P.hx, P.hy,
                         P.defect != 0, sd);
            if (P.qA) sd[0] += P.qA[cell];
            src[0] = (R)sd[0]; src[1] = (R)sd[1]; src[2] = (R)sd[2]; src[3] = (R)sd[3];
            R cf[4];
            cell_std<R>(d, src, (R)sigtA, xin, ydn, xo, yo, o, cf);
            if (P.psi && d.idx >= 0) {
#pragma unroll
              for (int m = 0; m < 4; ++m) P.psi[((long long)d.idx * 4 + m) * nc + cell] = (double)cf[m];
            }
          } else {
            double src = 0;
            if (P.x)
              src = lm_source<S == LMDG_SCHEME_RLMDG>(P.x, nc, cell, sxs, sys, c, jr, P.scatA[cell], P.absA[cell],
                                                      d.ox, d.oy, P.hx, P.hy, P.defect != 0);
            if (P.qA) src += P.qA[cell];
            R psi;
            if constexpr (S == LMDG_SCHEME_LMDG) {
              cell_lmdg<R>(d, (R)src, (R)sigtA, xin, ydn, xo, yo, o, psi);
            } else {
              const R kx = (c == 0) ? R(1) : R(0.5);
              cell_rlmdg<R>(d, (R)src, (R)sigtA, kx, ky, xin, ydn, xo, yo, o, psi);
            }
            if (P.psi && d.idx >= 0) P.psi[(long long)d.idx * nc + cell] = (double)psi;
          }
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) { xin[f] = xo[f]; yprev[f] = yo[f]; }
#pragma unroll
        for (int m = 0; m < NOUT; ++m) o[m] = quad_sum(o[m]);
        if (lane < 16) {
#pragma unroll
          for (int m = 0; m < NOUT; ++m) red[((tt * W + wv) * NOUT + m) * kRows + r] = o[m];
        }
        if (r == kRows - 1 && act && s + 1 < P.nstrips) {
          R* e = P.edge + ((((long long)q * P.nstrips + s) * nx + c) * NF) * P.dslots + slot;
#pragma unroll
          for (int f = 0; f < NF; ++f) store_agent(e + (long long)f * P.dslots, yo[f]);
        }
      }
      __syncthreads();
      // sums over waves, written with consecutive threads on consecutive columns
      const int nred = P.cw * NOUT * kRows;
      for (int e = tid; e < nred; e += blockDim.x) {
        const int tt = e % P.cw;
        const int m = (e / P.cw) % NOUT;
        const int rr = e / (P.cw * NOUT);
        const int c = t0 + tt - rr;
        const int jr2 = s * kRows + rr;
        if (jr2 < ny && c >= 0 && c < nx) {
          R acc = 0;
          for (int w2 = 0; w2 < W; ++w2) acc += red[((tt * W + w2) * NOUT + m) * kRows + rr];
          const int i = sxi > 0 ? c : nx - 1 - c;
          const int jj = syi > 0 ? jr2 : ny - 1 - jr2;
          P.part[((long long)q * NOUT + m) * nc + (long long)jj * nx + i] = acc;
        }
      }
      if (s + 1 < P.nstrips && tid == 0) {
        const int done = min(nx, t0 + P.cw - (kRows - 1));
        if (done > 0) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          store_agent(P.prog + (long long)q * P.nstrips + s, (P.epoch << 32) | (unsigned long long)done);
        }
      }
      __syncthreads();
    }
  }
}

template <typename R, int S>
int launch_typed(lmdg_handle* h, const double* x, bool use_q, double* psi, hipStream_t st, bool defect) {
  constexpr int NOUT = SchemeTraits<S>::NOUT;
  SweepParams<R> P;
  P.nx = (int)h->n[0];
  P.ny = (int)h->n[1];
  P.nstrips = h->nstrips;
  P.dslots = h->dslots;
  const int W = h->waves;
  int cw = 16;
  while (cw > 4 && (size_t)cw * W * NOUT * kRows * sizeof(R) > 64 * 1024) cw >>= 1;
  P.cw = cw;
  P.nchunks = (P.nx + kRows - 1 + cw - 1) / cw;
  P.n_items = 4 * h->nstrips;
  P.hx = h->h[0];
  P.hy = h->h[1];
  P.ncell = h->ncell;
  P.dirs = h->d_dirs;
  P.x = x;
  P.sigtA = h->d_sigtA;
  P.scatA = h->d_scatA;
  P.qA = use_q ? h->d_qA : nullptr;
  P.absA = h->d_absA;
  P.defect = defect ? 1 : 0;
  P.part = reinterpret_cast<R*>(h->ws.part);
  P.edge = reinterpret_cast<R*>(h->ws.edge);
  P.psi = psi;
  P.prog = h->ws.prog;
  P.ticket = h->ws.ticket;
  P.err = h->ws.err;
  P.epoch = h->epoch;
  P.ticket_base = h->ticket_base;
  const int grid = std::min(P.n_items, 4 * h->n_cu);
  const size_t lds = (size_t)cw * W * NOUT * kRows * sizeof(R);
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
  hipLaunchKernelGGL((sweep2d_kernel<R, S>), dim3(grid), dim3(64 * W), lds, st, P);
  if (ev_end) hipEventRecord(ev_end, st);
  h->epoch += 1;
  h->ticket_base += (unsigned)(P.n_items + grid);
  return check_hip(h, hipGetLastError(), "sweep launch");
}

}  // namespace

int launch_sweep(lmdg_handle* h, int scheme, int prec, const double* x, bool use_q, double* psi,
                 hipStream_t st, bool defect) {
  if (prec == LMDG_PREC_FP64) {
    switch (scheme) {
      case LMDG_SCHEME_STD: return launch_typed<double, LMDG_SCHEME_STD>(h, x, use_q, psi, st, defect);
      case LMDG_SCHEME_LMDG: return launch_typed<double, LMDG_SCHEME_LMDG>(h, x, use_q, psi, st, defect);
      default: return launch_typed<double, LMDG_SCHEME_RLMDG>(h, x, use_q, psi, st, defect);
    }
  }
  switch (scheme) {
    case LMDG_SCHEME_STD: return launch_typed<float, LMDG_SCHEME_STD>(h, x, use_q, psi, st, defect);
    case LMDG_SCHEME_LMDG: return launch_typed<float, LMDG_SCHEME_LMDG>(h, x, use_q, psi, st, defect);
    default: return launch_typed<float, LMDG_SCHEME_RLMDG>(h, x, use_q, psi, st, defect);
  }
}

}  // namespace lmdg
