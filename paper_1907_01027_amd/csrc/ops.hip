// Reductions into moment vectors, the B_11 stencil, and FP64 GMRES vector kernels.
#include "internal.h"

namespace lmdg {
namespace {

constexpr int kBlock = 256;

inline int grid_for(long long n, int per = kBlock) {
  long long g = (n + per - 1) / per;
  return (int)std::min<long long>(std::max<long long>(g, 1), 65535LL * 16);
}

// B_11 X_1 on one cell (Sec. 3.2, eq-lmdg-psi1, in the face form of Appendix C).
// Slopes u = a xi + b eta + c xi*eta are isotropic, so the streaming volume term
// sums to zero (condition (ii)) and only faces remain.  On a face with normal +e_k
// between K- and K+, directions with Omega_k > 0 take the trace of K-, the others
// that of K+; with c+ = sum_{Omega_k>0} w Omega_k and c- = sum_{Omega_k<0} w |Omega_k|
// the face contributes int (c+ u_- - c- u_+)(v_- - v_+).  The exterior trace is zero,
// which also covers boundary faces.  Mass term: eps sigma_a |K| diag(1/3, 1/3, 1/9).
__device__ __forceinline__ void b11_cell(const double* x, long long nc, int nx, int ny, int i, int j,
                                         double hx, double hy, double cxp, double cxm, double cyp,
                                         double cym, double absA, double& ya, double& yb, double& yc) {
  const long long p = (long long)j * nx + i;
  const double* xa = x + nc;
  const double* xb = x + 2 * nc;
  const double* xc = x + 3 * nc;
  const double a = xa[p], b = xb[p], c = xc[p];
  ya = absA * (1.0 / 3.0) * a;
  yb = absA * (1.0 / 3.0) * b;
  yc = absA * (1.0 / 9.0) * c;
  const double t3 = 1.0 / 3.0;
  {  // right face, K is the lower-x cell: trace a + (b + c) eta
    const bool in = i + 1 < nx;
    const double aR = in ? xa[p + 1] : 0.0, bR = in ? xb[p + 1] : 0.0, cR = in ? xc[p + 1] : 0.0;
    const double J0 = cxp * a + cxm * aR;
    const double J1 = cxp * (b + c) - cxm * (bR - cR);
    ya += hy * J0;
    yb += hy * J1 * t3;
    yc += hy * J1 * t3;
  }
  {  // left face, K is the upper-x cell: trace -a + (b - c) eta
    const bool in = i > 0;
    const double aL = in ? xa[p - 1] : 0.0, bL = in ? xb[p - 1] : 0.0, cL = in ? xc[p - 1] : 0.0;
    const double J0 = cxp * aL + cxm * a;
    const double J1 = cxp * (bL + cL) - cxm * (b - c);
    ya += hy * J0;
    yb -= hy * J1 * t3;
    yc += hy * J1 * t3;
  }
  {  // top face, K is the lower-y cell: trace b + (a + c) xi
    const bool in = j + 1 < ny;
    const double aT = in ? xa[p + nx] : 0.0, bT = in ? xb[p + nx] : 0.0, cT = in ? xc[p + nx] : 0.0;
    const double J0 = cyp * b + cym * bT;
    const double J1 = cyp * (a + c) - cym * (aT - cT);
    yb += hx * J0;
    ya += hx * J1 * t3;
    yc += hx * J1 * t3;
  }
  {  // bottom face, K is the upper-y cell: trace -b + (a - c) xi
    const bool in = j > 0;
    const double aB = in ? xa[p - nx] : 0.0, bB = in ? xb[p - nx] : 0.0, cB = in ? xc[p - nx] : 0.0;
    const double J0 = cyp * bB + cym * b;
    const double J1 = cyp * (aB + cB) - cym * (a - c);
    yb += hx * J0;
    ya -= hx * J1 * t3;
    yc += hx * J1 * t3;
  }
}

struct QuadMoments {
  double w[4], ax[4], ay[4];  // per quadrant: sum w, sum w |Omega_x|, sum w |Omega_y|
  int recon_y;                // 0 on slab handles: no reconstruction along y (see the sweep)
};

// G Sigma_0^T x_0: the second block row applied to the isotropic field x_0 copied to
// every direction (FP64, needed by the defect form of the operator).  Per direction
// the rows depend on Omega only through its quadrant and linearly through w,
// w|Omega_x|, w|Omega_y|, so the direction sum collapses to four quadrant terms.
// LMDG: G = Sigma L_10 (rows Ox h_y (u_up - u_K), Oy h_x (u_down - u_K), 0).
// RLMDG: G = Sigma (L_10 + L_11 R) - Sigma M_1 P_1 R, the rows of the sweep's cell
// formula evaluated with psi = x_0 everywhere (upwind slopes k (u - u_up), k = 1 in
// the inflow cell of the quadrant, traces zero outside the mesh).
template <bool RLM>
__device__ __forceinline__ void iso_g(const double* x0, int nx, int ny, int i, int j, double hx, double hy,
                                      double absA, const QuadMoments& qm, double g[3]) {
  auto val = [&](int ii, int jj) -> double {
    return (ii >= 0 && ii < nx && jj >= 0 && jj < ny) ? x0[(long long)jj * nx + ii] : 0.0;
  };
  const double v = x0[(long long)j * nx + i];
  const double t3 = 1.0 / 3.0;
  g[0] = g[1] = g[2] = 0.0;
  for (int q = 0; q < 4; ++q) {
    const int sx = (q & 1) ? -1 : 1, sy = (q & 2) ? -1 : 1;
    const double W = qm.w[q], AX = qm.ax[q], AY = qm.ay[q];
    const bool upx = sx > 0 ? i > 0 : i < nx - 1;  // upwind x neighbour inside the mesh
    const bool upy = sy > 0 ? j > 0 : j < ny - 1;
    const double u1 = val(i - sx, j), d1 = val(i, j - sy);
    if (!RLM) {
      g[0] += sx * AX * hy * (u1 - v);
      g[1] += sy * AY * hx * (d1 - v);
      continue;
    }
    const double u2 = val(i - 2 * sx, j), d2 = val(i, j - 2 * sy), ud = val(i - sx, j - sy);
    const double kx = upx ? 0.5 : 1.0, ky = qm.recon_y ? (upy ? 0.5 : 1.0) : 0.0;
    // is the upwind neighbour itself the inflow cell of its line?
    const double kxu = (sx > 0 ? i - 1 == 0 : i + 1 == nx - 1) ? 1.0 : 0.5;
    const double kyd = (sy > 0 ? j - 1 == 0 : j + 1 == ny - 1) ? 1.0 : 0.5;
    const double cxi = sx * kx * (v - u1);
    const double ceta = sy * ky * (v - d1);
    const double txu = upx ? u1 + kxu * (u1 - u2) : 0.0;
    const double tyd = upy ? d1 + kyd * (d1 - d2) : 0.0;
    const double cxi_d = upy ? sx * kx * (d1 - ud) : 0.0;    // xi slope of the cell below
    const double ceta_u = upx ? sy * ky * (u1 - ud) : 0.0;   // eta slope of the cell on the left
    // slope mass terms: sigma_t|K|/3 of L_11 R minus (sigma_s/eps)|K|/3 of M_1 P_1 R
    g[0] += sx * AX * hy * (txu - v) + (absA * t3 * W + AX * hy + AY * hx * t3) * cxi - AY * hx * t3 * cxi_d;
    g[1] += sy * AY * hx * (tyd - v) + (absA * t3 * W + AY * hx + AX * hy * t3) * ceta - AX * hy * t3 * ceta_u;
    g[2] += t3 * (sx * AX * hy * (ceta_u - ceta) + sy * AY * hx * (cxi_d - cxi));
  }
}

// Reduced operator / right-hand side / recovery for LMDG and RLMDG from the
// per-quadrant sweep sums (eq-nonrec-block; Sec. 3.3.2 with the second block row
// G = Sigma (L_10 + L_11 R) - Sigma M_1 P_1 R).  In kApplyDefect the sweep solved
// L~_00 psi_D = defect source, and K x = [P_0 psi_D ; B_11 x_1 - G Sigma_0^T x_0 + G psi_D].
//
// Source data.  With F(x) = [x_0 - P_0 psi ; B_11 x_1 - G psi], psi the sweep of x with
// the source and the inflow data (taken as ghost traces upwind of the inflow faces),
// the isotropic test functions of the slope rows give F(x) = [0 ; -Sigma Q_1^q] with
// x_1 = -(Phi_1 - P_1 R Psi_0) (LMDG: -Phi_1), Sigma Q_1^q the direction sum of the
// source slope moments: the inflow part of Sigma Q_1 is carried by the ghost traces
// (for LMDG only its face averages; sqa holds the rest).  So K x = b with
// b = -F(0) - [0 ; sq1 + sqa]: the right-hand-side sweep (x = 0) minus the
// corrections, and recovery Phi_1 = -x_1 + P_1 R Psi_0 needs no c.
template <typename R, bool RLM>
__global__ void combine_lm_kernel(int mode, int nr, int nsl, int nx, int ny, double hx, double hy, double cxp, double cxm,
                                  double cyp, double cym, QuadMoments qm, const double* __restrict__ x_all,
                                  const R* __restrict__ part_all, const double* __restrict__ absA,
                                  const double* __restrict__ sq1, const double* __restrict__ sqa,
                                  double* __restrict__ out_all) {
  constexpr int NOUT = RLM ? 6 : 3;
  const long long nc = (long long)nx * ny;
  for (long long pr = blockIdx.x * (long long)blockDim.x + threadIdx.x; pr < nr * nc;
       pr += (long long)gridDim.x * blockDim.x) {
    // right-hand side rh, cell p; vectors are stacked rhs-major
    const long long rh = pr / nc, p = pr - rh * nc;
    const double* x = x_all ? x_all + rh * 4 * nc : nullptr;
    const R* part = part_all + rh * nsl * NOUT * nc;
    double* out = out_all + rh * 4 * nc;
    // rows the mode reads (RLMDG sweeps produce the P_1 R rows for the recovery only)
    double s[NOUT];
#pragma unroll
    for (int m = 0; m < NOUT; ++m) {
      double acc = 0;
      if (!RLM || m < 4 || mode == kRecover)
        for (int q = 0; q < nsl; ++q) acc += (double)part[((long long)q * NOUT + m) * nc + p];
      s[m] = acc;
    }
    // the sweep's slope rows already hold G Psi (with Sigma M_1 P_1 R taken per direction)
    const double g1 = s[1], g2 = s[2];
    const double g3 = RLM ? s[3] : 0.0;
    if (mode == kApply) {
      const int i = (int)(p % nx), j = (int)(p / nx);
      double ya, yb, yc;
      b11_cell(x, nc, nx, ny, i, j, hx, hy, cxp, cxm, cyp, cym, absA[p], ya, yb, yc);
      out[p] = x[p] - s[0];
      out[nc + p] = ya - g1;
      out[2 * nc + p] = yb - g2;
      out[3 * nc + p] = yc - g3;
    } else if (mode == kApplyDefect) {
      const int i = (int)(p % nx), j = (int)(p / nx);
      double ya, yb, yc, gi[3];
      b11_cell(x, nc, nx, ny, i, j, hx, hy, cxp, cxm, cyp, cym, absA[p], ya, yb, yc);
      iso_g<RLM>(x, nx, ny, i, j, hx, hy, absA[p], qm, gi);
      out[p] = s[0];
      out[nc + p] = ya - gi[0] + g1;
      out[2 * nc + p] = yb - gi[1] + g2;
      out[3 * nc + p] = yc - gi[2] + g3;
    } else if (mode == kRhs) {
      double c1 = 0.0, c2 = 0.0, c3 = 0.0;
      if (sq1) { c1 += sq1[p]; c2 += sq1[nc + p]; c3 += sq1[2 * nc + p]; }
      if (sqa) { c1 += sqa[p]; c2 += sqa[nc + p]; c3 += sqa[2 * nc + p]; }
      out[p] = s[0];
      out[nc + p] = g1 - c1;
      out[2 * nc + p] = g2 - c2;
      out[3 * nc + p] = g3 - c3;
    } else {  // recovery: Phi_1 = -X_1 + P_1 R Psi_0
      out[p] = s[0];
      out[nc + p] = -x[nc + p] + (RLM ? s[4] : 0.0);
      out[2 * nc + p] = -x[2 * nc + p] + (RLM ? s[5] : 0.0);
      out[3 * nc + p] = -x[3 * nc + p];
    }
  }
}

// Standard scheme: K Phi = Phi - P L^{-1} M Phi (eq-sndg-phi); right-hand side and
// recovered scalar flux are the plain quadrant sums.
template <typename R>
__global__ void combine_std_kernel(int mode, int nr, int nsl, int np, long long nc, const double* __restrict__ x_all,
                                   const R* __restrict__ part_all, double* __restrict__ out_all) {
  for (long long pr = blockIdx.x * (long long)blockDim.x + threadIdx.x; pr < nr * nc;
       pr += (long long)gridDim.x * blockDim.x) {
    const long long rh = pr / nc, p = pr - rh * nc;
    const double* x = x_all ? x_all + rh * np * nc : nullptr;
    const R* part = part_all + rh * nsl * np * nc;
    double* out = out_all + rh * np * nc;
    for (int m = 0; m < np; ++m) {
      double acc = 0;
      for (int q = 0; q < nsl; ++q) acc += (double)part[((long long)q * np + m) * nc + p];
      // kApplyDefect: the sweep already produced P L^{-1}(defect source) = K Phi
      out[m * nc + p] = (mode == kApply) ? x[m * nc + p] - acc : acc;
    }
  }
}

template <typename R>
__global__ void sum_quadrants_kernel(int nout, int nout_abi, int nr, int nsl, long long nc, const R* __restrict__ part_all,
                                     double* __restrict__ out_all) {
  for (long long pr = blockIdx.x * (long long)blockDim.x + threadIdx.x; pr < nr * nc;
       pr += (long long)gridDim.x * blockDim.x) {
    const long long rh = pr / nc, p = pr - rh * nc;
    const R* part = part_all + rh * nsl * nout * nc;
    double* out = out_all + rh * nout_abi * nc;
    for (int m = 0; m < nout_abi; ++m) {
      double acc = 0;
      if (m < nout)
        for (int q = 0; q < nsl; ++q) acc += (double)part[((long long)q * nout + m) * nc + p];
      out[m * nc + p] = acc;
    }
  }
}

// y = [0 ; B_11 x_1] on the moment-major layout (slot 0 of x is not read).
__global__ void b11_apply_kernel(int nx, int ny, double hx, double hy, double cxp, double cxm, double cyp,
                                 double cym, const double* __restrict__ x, const double* __restrict__ absA,
                                 double* __restrict__ y) {
  const long long nc = (long long)nx * ny;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < nc;
       p += (long long)gridDim.x * blockDim.x) {
    double ya, yb, yc;
    b11_cell(x, nc, nx, ny, (int)(p % nx), (int)(p / nx), hx, hy, cxp, cxm, cyp, cym, absA[p], ya, yb, yc);
    y[p] = 0.0;
    y[nc + p] = ya;
    y[2 * nc + p] = yb;
    y[3 * nc + p] = yc;
  }
}

// Gradients of J = int phi d with respect to per-cell sigma_s, sigma_a, q from the
// forward angular flux psi and the adjoint angular flux lambda (bilinear form of
// eq-Ljk differentiated cell by cell):
//   dJ/dsigma_a = -eps sum_l w_l int_K psi_l lambda_l
//   dJ/dsigma_s = -(1/eps) (sum_l w_l int_K psi_l lambda_l - int_K phi Lambda)
//   dJ/dq       =  eps int_K Lambda
// with phi, Lambda the scalar fluxes.  The adjoint field of direction l is the
// forward-type solution of direction -Omega_l.  The direction sum is accumulated one
// quadrant at a time from that quadrant's forward fluxes and the opposite quadrant's
// adjoint-type fluxes, both indexed by direction slot (pairs: w_l and the slot of
// -Omega_l); npsi = 4 (standard: all moments per direction) or 1 (low-memory: Psi_0
// per direction, the slope part being the isotropic Phi_1 of phi / Lambda).  Legendre
// mass on K is |K| diag(1, 1/3, 1/3, 1/9).
__global__ void grad_accum_kernel(long long nc, int dslots, int npsi, const double* __restrict__ pairs,
                                  const double* __restrict__ psi, const double* __restrict__ lam,
                                  double* __restrict__ bil) {
  const double mass[4] = {1.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 9.0};
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < nc;
       p += (long long)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int k = 0; k < dslots; ++k) {
      const double w = pairs[2 * k];
      const long long kn = (long long)pairs[2 * k + 1];
      double a = 0.0;
      for (int m = 0; m < npsi; ++m)
        a += mass[m] * psi[((long long)k * npsi + m) * nc + p] * lam[(kn * npsi + m) * nc + p];
      acc += w * a;
    }
    bil[p] += acc;
  }
}

__global__ void grad_final_kernel(long long nc, int npsi, const double* __restrict__ bil_in,
                                  const double* __restrict__ phi, const double* __restrict__ Lam,
                                  const double* __restrict__ epsA, double area, double* __restrict__ gs,
                                  double* __restrict__ ga, double* __restrict__ gq) {
  const double mass[4] = {1.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 9.0};
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < nc;
       p += (long long)gridDim.x * blockDim.x) {
    double bil = bil_in[p];
    double bar = 0.0, slopes = 0.0;
    for (int m = 0; m < 4; ++m) {
      const double t = mass[m] * phi[m * nc + p] * Lam[m * nc + p];
      bar += t;
      if (m > 0) slopes += t;
    }
    if (npsi == 1) bil += slopes;  // isotropic slope part, sum_l w_l = 1
    const double eA = epsA[p];
    const double eps = eA / area;
    ga[p] = -eA * bil;
    gs[p] = -(area / eps) * (bil - bar);
    gq[p] = eA * Lam[p];
  }
}

// Source of the adjoint RLMDG sweep, per direction and cell (unweighted rows).
//
// The adjoint of the Petrov-Galerkin system A = T^T (L - M P) T_R (eq-rlmdg-vari) is
// A^T lambda = j.  With the directions reflected (on a centrally symmetric set L_l^T is
// L_{-l} and M P is symmetric), it becomes the Petrov-Galerkin system with trial space T
// (cell constants per direction plus isotropic slopes) and test space T_R', R' the
// downwind reconstruction (the upwind one of -Omega).  Testing with the slope part of
// T_R' and using the isotropic slope rows to remove the P_1^T Sigma part, the constant
// rows of direction l read
//   (L_00 + R'^T L_10) mu_l = M_0 X_0 + L_01 X'_1 + R'^T ((L_11 - M_1) X'_1 + d_1) + d_0,
// with X_0 = P_0 mu, X'_1 = -(the isotropic slopes), d = the detector moments, and the
// slope rows give B_11 X'_1 - Sigma L_10 mu = -d_1.  L_00 + R'^T L_10 has the stencil of
// the forward L~_00 with k = 1 in the outflow cell of a line and 1/2 elsewhere, so the
// RLMDG sweep solves it with those rules; this kernel forms the right-hand side.
// R'^T of a slope-row field rho: sum over axes a of s_a (-k_a(K) rho_a(K) +
// k_a(U_a) rho_a(U_a)), U_a the upwind neighbour (k = 1/2 there: K is downwind of it);
// rho_xi(J) = (eps sigma_a|J|/3 + ax + ay/3) a_J + ay s_y c_J / 3 + ax a_{U_x(J)}
//             - ay (a_{U_y(J)} + s_y c_{U_y(J)}) / 3 + d_xi(J)   (and eta with x <-> y),
// (a, b, c) the xi, eta, xi eta coefficients of X'_1, ax = |Ox| h_y, ay = |Oy| h_x; the
// scattering parts of L_11 and M_1 cancel to eps sigma_a.
__global__ void adj_rlm_source_kernel(int nx, int ny, double hx, double hy, int dslots, int recon_y,
                                      const double* __restrict__ dirs, const double* __restrict__ x,
                                      const double* __restrict__ det, const double* __restrict__ scatA,
                                      const double* __restrict__ absA, double* __restrict__ out) {
  const long long nc = (long long)nx * ny;
  const long long total = 4LL * dslots * nc;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long p = e % nc;
    const int qs = (int)(e / nc);  // quadrant * dslots + slot
    const double* dr = dirs + (long long)qs * kDirStride;
    const int l = (int)dr[3];
    if (l < 0) continue;
    const int q = qs / dslots;
    const int sx = (q & 1) ? -1 : 1, sy = (q & 2) ? -1 : 1;
    const double ox = dr[0], oy = dr[1];
    const double ax = fabs(ox) * hy, ay = fabs(oy) * hx;
    const int i = (int)(p % nx), j = (int)(p / nx);
    // value of moment r of (x or det) at cell (ii, jj); zero outside
    auto v = [&](const double* f, int r, int ii, int jj) -> double {
      if (!f || ii < 0 || ii >= nx || jj < 0 || jj >= ny) return 0.0;
      return f[(long long)r * nc + (long long)jj * nx + ii];
    };
    auto rho_xi = [&](int ii, int jj) -> double {
      const double a = v(x, 1, ii, jj), c = v(x, 3, ii, jj);
      const double aux = v(x, 1, ii - sx, jj);
      const double auy = v(x, 1, ii, jj - sy), cuy = v(x, 3, ii, jj - sy);
      const double aA = absA[(long long)jj * nx + ii];
      return (aA / 3.0 + ax + ay / 3.0) * a + ay * sy * c / 3.0 + ax * aux - ay * (auy + sy * cuy) / 3.0 +
             v(det, 1, ii, jj);
    };
    auto rho_eta = [&](int ii, int jj) -> double {
      const double b = v(x, 2, ii, jj), c = v(x, 3, ii, jj);
      const double buy = v(x, 2, ii, jj - sy);
      const double bux = v(x, 2, ii - sx, jj), cux = v(x, 3, ii - sx, jj);
      const double aA = absA[(long long)jj * nx + ii];
      return (aA / 3.0 + ay + ax / 3.0) * b + ax * sx * c / 3.0 + ay * buy - ax * (bux + sx * cux) / 3.0 +
             v(det, 2, ii, jj);
    };
    const bool upx = sx > 0 ? i > 0 : i < nx - 1, upy = sy > 0 ? j > 0 : j < ny - 1;
    const bool outx = sx > 0 ? i == nx - 1 : i == 0, outy = sy > 0 ? j == ny - 1 : j == 0;
    const double kx = outx ? 1.0 : 0.5, ky = outy ? 1.0 : 0.5;
    double src = scatA[p] * v(x, 0, i, j) + v(det, 0, i, j);
    // L_01 X'_1: outflow traces of the slopes minus the inflow ones
    src += ox * hy * (v(x, 1, i, j) - v(x, 1, i - sx, j)) + oy * hx * (v(x, 2, i, j) - v(x, 2, i, j - sy));
    // R'^T rho
    double rt = sx * (-kx * rho_xi(i, j) + (upx ? 0.5 * rho_xi(i - sx, j) : 0.0));
    if (recon_y) rt += sy * (-ky * rho_eta(i, j) + (upy ? 0.5 * rho_eta(i, j - sy) : 0.0));
    out[(long long)l * nc + p] = src + rt;
  }
}

// ---------------------------------------------------------------- GMRES vectors
constexpr int kDotBlocks = 240;

// Vectors of nr right-hand sides are stacked (segments of length n).  For the group of
// up to kDotGroup basis vectors v0 + 0.. (blockIdx.y) and segment rz (blockIdx.z):
// partial[(v * nr + rz) * kDotBlocks + b] = block b's share of V_v[rz] . w[rz]; each
// element of w is read once per group.
// The basis may be stored in FP32 (TV = float: the inner solves of mode MIXED); products
// and sums are FP64.
constexpr int kDotGroup = 8;
template <typename TV>
__global__ void dots_partial_kernel(const TV* __restrict__ V, long long ld, int nvec,
                                    const double* __restrict__ w_all, long long n, double* __restrict__ partial) {
  const int v0 = blockIdx.y * kDotGroup;
  const int nv = min(kDotGroup, nvec - v0);
  const int rz = blockIdx.z;
  const double* w = w_all + rz * n;
  double acc[kDotGroup];
#pragma unroll
  for (int k = 0; k < kDotGroup; ++k) acc[k] = 0.0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const double we = w[e];
#pragma unroll
    for (int k = 0; k < kDotGroup; ++k)
      if (k < nv) acc[k] += (double)V[(v0 + k) * ld + rz * n + e] * we;
  }
  __shared__ double sh[kDotGroup][kBlock];
#pragma unroll
  for (int k = 0; k < kDotGroup; ++k) sh[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s2 = kBlock / 2; s2 > 0; s2 >>= 1) {
    if (threadIdx.x < s2)
#pragma unroll
      for (int k = 0; k < kDotGroup; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s2];
    __syncthreads();
  }
  if (threadIdx.x < nv)
    partial[((long long)(v0 + threadIdx.x) * gridDim.z + rz) * gridDim.x + blockIdx.x] = sh[threadIdx.x][0];
}

__global__ void dots_final_kernel(const double* __restrict__ partial, int nparts, double* __restrict__ out) {
  const int v = blockIdx.x;
  __shared__ double sh[kBlock];
  double acc = 0;
  for (int e = threadIdx.x; e < nparts; e += blockDim.x) acc += partial[(long long)v * nparts + e];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = sh[0];
}

// w[rz] += sign * sum_v coef[v * nr + rz] V_v[rz] over stacked segments of length n
template <typename TV>
__global__ void axpy_multi_kernel(double* __restrict__ w, const TV* __restrict__ V, long long ld, int nvec,
                                  const double* __restrict__ coef, double sign, long long n, int nr) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n * nr;
       e += (long long)gridDim.x * blockDim.x) {
    const long long rz = e / n;
    double acc = 0;
    for (int v = 0; v < nvec; ++v) acc += coef[(long long)v * nr + rz] * (double)V[v * ld + e];
    w[e] += sign * acc;
  }
}

// y[rz] = scale[rz] * x[rz] over stacked segments of length n (scale on the device),
// rounded to the type of y
template <typename TY>
__global__ void scale_seg_kernel(TY* __restrict__ y, const double* __restrict__ x,
                                 const double* __restrict__ scale, long long n, int nr) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n * nr;
       e += (long long)gridDim.x * blockDim.x)
    y[e] = (TY)(scale[e / n] * x[e]);
}

__global__ void widen_kernel(double* __restrict__ y, const float* __restrict__ x, long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    y[e] = (double)x[e];
}

__global__ void axpby_kernel(double* __restrict__ y, double a, const double* __restrict__ x, double b,
                             long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    y[e] = (b == 0.0) ? a * x[e] : a * x[e] + b * y[e];  // b = 0 never reads y
}

__global__ void fill_kernel(double* __restrict__ y, double v, long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    y[e] = v;
}

}  // namespace

int dots_partials() { return kDotBlocks; }

void launch_combine(lmdg_handle* h, int scheme, int prec, int mode, const double* x, double* out,
                    hipStream_t st) {
  if (h->dim == 3 && scheme != LMDG_SCHEME_STD) {
    launch_combine3(h, scheme, prec, mode, x, out, st);
    return;
  }
  const long long nc = h->ncell;
  const int nr = h->n_rhs;
  const int g = std::min(grid_for(nc * nr), 4096);
  const int nx = (int)h->n[0], ny = (int)h->n[1];
  if (scheme == LMDG_SCHEME_STD) {
    // 3D: the plain form (one slice per octant of the eight moments)
    if (prec == LMDG_PREC_FP64)
      hipLaunchKernelGGL(combine_std_kernel<double>, dim3(g), dim3(kBlock), 0, st, mode, nr, h->last_nsl, h->np, nc,
                         x, (const double*)h->ws.part, out);
    else
      hipLaunchKernelGGL(combine_std_kernel<float>, dim3(g), dim3(kBlock), 0, st, mode, nr, h->last_nsl, h->np, nc, x,
                         (const float*)h->ws.part, out);
    return;
  }
  const double hx = h->h[0], hy = h->h[1];
  QuadMoments qm;
  qm.recon_y = h->slab ? 0 : 1;
  for (int q = 0; q < 4; ++q) {
    qm.w[q] = h->qw[q];
    qm.ax[q] = h->qax[q];
    qm.ay[q] = h->qay[q];
  }
#define LMDG_COMBINE(R, RLM)                                                                        \
  hipLaunchKernelGGL((combine_lm_kernel<R, RLM>), dim3(g), dim3(kBlock), 0, st, mode, nr, h->last_nsl, nx, ny, hx, hy, \
                     h->cplus[0], h->cminus[0], h->cplus[1], h->cminus[1], qm, x,                    \
                     (const R*)h->ws.part, h->d_absA, sq1, sqa, out)
  const bool rlm = scheme == LMDG_SCHEME_RLMDG;
  // right-hand-side corrections of the handle's own source data (not of an adjoint source)
  const bool own = mode == kRhs && !h->src0;
  const double* sq1 = own ? h->d_sq1 : nullptr;
  const double* sqa = (own && !rlm) ? h->d_sqa : nullptr;
  if (h->adj_rlm) {  // adjoint of RLMDG: right-hand side minus the detector's slope moments
    sq1 = mode == kRhs ? h->adj_det + nc : nullptr;
    sqa = nullptr;
  }
  if (prec == LMDG_PREC_FP64) {
    if (rlm) LMDG_COMBINE(double, true); else LMDG_COMBINE(double, false);
  } else {
    if (rlm) LMDG_COMBINE(float, true); else LMDG_COMBINE(float, false);
  }
#undef LMDG_COMBINE
}

void launch_sum_quadrants(lmdg_handle* h, int scheme, int prec, double* out, hipStream_t st) {
  if (h->dim == 3 && scheme != LMDG_SCHEME_STD) {
    launch_sum_octants(h, scheme, prec, out, st);
    return;
  }
  const int nout = scheme == LMDG_SCHEME_STD ? h->np : (scheme == LMDG_SCHEME_LMDG ? 3 : 6);
  const int nout_abi = scheme == LMDG_SCHEME_RLMDG ? 6 : h->np;
  const int g = std::min(grid_for(h->ncell * h->n_rhs), 4096);
  if (prec == LMDG_PREC_FP64)
    hipLaunchKernelGGL(sum_quadrants_kernel<double>, dim3(g), dim3(kBlock), 0, st, nout, nout_abi, h->n_rhs,
                       h->last_nsl, h->ncell, (const double*)h->ws.part, out);
  else
    hipLaunchKernelGGL(sum_quadrants_kernel<float>, dim3(g), dim3(kBlock), 0, st, nout, nout_abi, h->n_rhs,
                       h->last_nsl, h->ncell, (const float*)h->ws.part, out);
}

void launch_adj_rlm_source(lmdg_handle* h, const double* x, const double* det, hipStream_t st) {
  const int g = std::min(grid_for(4LL * h->dslots * h->ncell), 8192);
  hipLaunchKernelGGL(adj_rlm_source_kernel, dim3(g), dim3(kBlock), 0, st, (int)h->n[0], (int)h->n[1], h->h[0],
                     h->h[1], h->dslots, h->slab ? 0 : 1, h->d_dirs, x, det, h->d_scatA, h->d_absA, h->d_adjsrc);
}

void launch_b11(lmdg_handle* h, const double* x, double* y, hipStream_t st) {
  if (h->dim == 3) {
    launch_b11_3d(h, x, y, st);
    return;
  }
  const int g = std::min(grid_for(h->ncell), 4096);
  hipLaunchKernelGGL(b11_apply_kernel, dim3(g), dim3(kBlock), 0, st, (int)h->n[0], (int)h->n[1], h->h[0], h->h[1],
                     h->cplus[0], h->cminus[0], h->cplus[1], h->cminus[1], x, h->d_absA, y);
}

void launch_grad_accumulate(lmdg_handle* h, int quadrant, int npsi, double* bil, hipStream_t st) {
  const int g = std::min(grid_for(h->ncell), 4096);
  hipLaunchKernelGGL(grad_accum_kernel, dim3(g), dim3(kBlock), 0, st, h->ncell, h->dslots, npsi,
                     h->d_adjpairs + (size_t)quadrant * h->dslots * 2, h->d_psi_f, h->d_psi_a, bil);
}

void launch_gradients(lmdg_handle* h, int npsi, const double* bil, const double* phi, const double* Lam, double* gs,
                      double* ga, double* gq, hipStream_t st) {
  const int g = std::min(grid_for(h->ncell), 4096);
  hipLaunchKernelGGL(grad_final_kernel, dim3(g), dim3(kBlock), 0, st, h->ncell, npsi, bil, phi, Lam, h->d_epsA,
                     h->area, gs, ga, gq);
}

template <typename TV>
static void dots_impl(const TV* V, long long ld, int nvec, const double* w, long long n, double* partial, double* out,
                      hipStream_t st, int nr) {
  hipLaunchKernelGGL(dots_partial_kernel<TV>, dim3(kDotBlocks, (nvec + kDotGroup - 1) / kDotGroup, nr), dim3(kBlock),
                     0, st, V, ld, nvec, w, n, partial);
  hipLaunchKernelGGL(dots_final_kernel, dim3(nvec * nr), dim3(kBlock), 0, st, partial, kDotBlocks, out);
}
void vec_dots(const double* V, long long ld, int nvec, const double* w, long long n, double* partial,
              double* out, hipStream_t st, int nr) {
  dots_impl(V, ld, nvec, w, n, partial, out, st, nr);
}
void vec_dots(const float* V, long long ld, int nvec, const double* w, long long n, double* partial,
              double* out, hipStream_t st, int nr) {
  dots_impl(V, ld, nvec, w, n, partial, out, st, nr);
}

void vec_scale_seg(double* y, const double* x, const double* scale, long long n, int nr, hipStream_t st) {
  hipLaunchKernelGGL(scale_seg_kernel<double>, dim3(std::min(grid_for(n * nr), 4096)), dim3(kBlock), 0, st, y, x,
                     scale, n, nr);
}
void vec_scale_seg(float* y, const double* x, const double* scale, long long n, int nr, hipStream_t st) {
  hipLaunchKernelGGL(scale_seg_kernel<float>, dim3(std::min(grid_for(n * nr), 4096)), dim3(kBlock), 0, st, y, x,
                     scale, n, nr);
}

void vec_axpy_multi(double* w, const double* V, long long ld, int nvec, const double* coef, double sign,
                    long long n, hipStream_t st, int nr) {
  hipLaunchKernelGGL(axpy_multi_kernel<double>, dim3(std::min(grid_for(n * nr), 4096)), dim3(kBlock), 0, st, w, V,
                     ld, nvec, coef, sign, n, nr);
}
void vec_axpy_multi(double* w, const float* V, long long ld, int nvec, const double* coef, double sign,
                    long long n, hipStream_t st, int nr) {
  hipLaunchKernelGGL(axpy_multi_kernel<float>, dim3(std::min(grid_for(n * nr), 4096)), dim3(kBlock), 0, st, w, V,
                     ld, nvec, coef, sign, n, nr);
}

void vec_widen(double* y, const float* x, long long n, hipStream_t st) {
  hipLaunchKernelGGL(widen_kernel, dim3(std::min(grid_for(n), 4096)), dim3(kBlock), 0, st, y, x, n);
}

void vec_axpby(double* y, double a, const double* x, double b, long long n, hipStream_t st) {
  hipLaunchKernelGGL(axpby_kernel, dim3(std::min(grid_for(n), 4096)), dim3(kBlock), 0, st, y, a, x, b, n);
}

void vec_copy(double* y, const double* x, long long n, hipStream_t st) {
  hipMemcpyAsync(y, x, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st);
}

void vec_fill(double* y, double v, long long n, hipStream_t st) {
  hipLaunchKernelGGL(fill_kernel, dim3(std::min(grid_for(n), 4096)), dim3(kBlock), 0, st, y, v, n);
}

}  // namespace lmdg
