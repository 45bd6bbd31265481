// Two-level right preconditioner of the reduced LMDG / RLMDG systems (2D).
//
// The paper leaves preconditioning of the dimension-reduced system open (Sec. 5, item
// (ii)) and derives the eps -> 0 limit of the low-memory scheme in Sec. 3.1: continuous
// Q^1 functions with cell-averaged gradients (eq-difflimPF).  The library applies
//
//     M^{-1} r = K_loc^{-1} r + Z B^{-1} W r
//
// * K_loc: the 4 x 4 diagonal block of K of every cell (rows and columns X_0, X_1 of that
//   cell), in closed form: K_loc = diag(1, B_11|KK) - sum_l [w_l ; g_l] a_l^{-1} [m_l, u_l],
//   with a_l the local sweep diagonal (sigma_t |K| + |Omega_x| h_y (1 + k_x) + |Omega_y| h_x
//   (1 + k_y), k = 0 for LMDG, 1/2 or 1 in the inflow cell for RLMDG), m_l = (sigma_s/eps)|K|,
//   u_l = (Omega_x h_y, Omega_y h_x, 0) the cell's own slope terms of the sweep source and g_l
//   the cell's own coefficient in the slope rows of the angular sum (eq-nonrec-block, and
//   for RLMDG the corrected second block row Sigma L_10 + Sigma L_11 R - Sigma M_1 P_1 R).
//   The cell-average row is formed as sum_l w_l (a_l - m_l) / a_l so that no O(sigma_s/eps)
//   terms cancel.
// * W: the residual as a source of the full scheme (cell moments (sigma_s/eps) r_0 and
//   -r_m / (|K| n_m)) loaded onto nodal Q^1 functions: f_c = sum_K (1/4)[(sigma_s/eps)|K| r_0
//   - c_x r_xi - c_y r_eta - c_x c_y r_xieta], (c_x, c_y) = (+-1, +-1) the corner of K.
// * B: eq-difflimPF with coefficient D = 1/(3 sigma_t) and absorption eps sigma_a, plus
//   1/2 int_{dD} u v, mass and boundary terms lumped, keeping only the couplings between
//   nodes of equal parity of i + j (all of them on square cells): per cell the diagonal
//   (SW, NE) and (SE, NW) node pairs are joined with the weight D |K| (1/(4 h_x^2) +
//   1/(4 h_y^2)).  The two parity classes are two independent systems ("colours").
// * Z: nodal u -> cell Legendre moments [avg ; -xi ; -eta ; -xieta], and for RLMDG plus the
//   angular average of the reconstructed slopes of the isotropic cell averages.
//
// B^{-1} is applied by V-cycles of a geometric multigrid per colour.  Level 0 is the
// colour's node sublattice (diagonal couplings only, bipartite by the parity of j, so a
// two-colour Gauss-Seidel sweep is exact Gauss-Seidel).  Level 1 is the Cartesian grid of
// the nodes with i and j even for both colours: colour 0 (i + j even) injects there and
// averages the four diagonal neighbours at nodes with i, j odd; colour 1 (i + j odd)
// averages the two axial neighbours.  Further levels coarsen a Cartesian grid to its even
// nodes with (boundary-normalised) bilinear interpolation and four-colour Gauss-Seidel on
// the 9-point Galerkin operators P^T A P, computed on the GPU from the level above; the
// coarsest grid (at most kCoarseMax nodes) is solved with its dense inverse.  A fixed number
// of V-cycles from zero is a fixed linear map, so plain right-preconditioned GMRES applies.
#include "internal.h"

#include <algorithm>
#include <cmath>

namespace lmdg {
namespace {

constexpr int kT = 256;
constexpr int kCoarseMax = 128;   // nodes of the coarsest grid (dense inverse)

inline int blocks_for(long long n) { return (int)std::max<long long>(1, (n + kT - 1) / kT); }

struct Geo {
  int nx, ny, NX, NY;   // cells and nodes per axis
  long long ncell;
  double hx, hy, area;
};

__device__ __forceinline__ double sgnd(double v) { return v > 0.0 ? 1.0 : -1.0; }

// ---------------------------------------------------------------- cell blocks K_loc^{-1}
__global__ void kloc_kernel(Geo g, const double* __restrict__ dirs, int nslots, const double* __restrict__ sigtA,
                            const double* __restrict__ scatA, const double* __restrict__ absA, double cxp,
                            double cxm, double cyp, double cym, int rlm, double* __restrict__ kinv) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.ncell) return;
  const int i = (int)(p % g.nx), j = (int)(p / g.nx);
  const double st = sigtA[p], sc = scatA[p], ab = absA[p];
  double K[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) K[a][b] = 0.0;
  for (int s = 0; s < nslots; ++s) {
    const double* d = dirs + (size_t)s * kDirStride;
    const double w = d[2];
    if (w == 0.0) continue;  // padding slot
    const double ox = d[0], oy = d[1];
    const double ax = fabs(ox) * g.hy, ay = fabs(oy) * g.hx;
    const double sx = sgnd(ox), sy = sgnd(oy);
    double kx = 0.0, ky = 0.0;
    if (rlm) {  // reconstruction factor: 1 in the inflow cell along the axis, 1/2 inside
      kx = (sx > 0.0 ? i == 0 : i == g.nx - 1) ? 1.0 : 0.5;
      ky = (sy > 0.0 ? j == 0 : j == g.ny - 1) ? 1.0 : 0.5;
    }
    const double fx = ax * (1.0 + kx), fy = ay * (1.0 + ky);
    const double ia = 1.0 / (st + fx + fy);
    const double amm = ab + fx + fy;  // a_l - (sigma_s/eps)|K|
    const double u0 = ox * g.hy, u1 = oy * g.hx;
    double g0 = -ox * g.hy, g1 = -oy * g.hx, g2 = 0.0;
    if (rlm) {
      // own slope-row coefficients of Sigma L_11 R - Sigma M_1 P_1 R: L_11 of the cell with
      // the scattering part of its mass removed (eps sigma_a |K| diag(1/3, 1/3, 1/9)),
      // applied to the reconstructed slopes (s_x k_x, s_y k_y, 0) per unit psi_K
      g0 += (ax + ay * (1.0 / 3.0) + ab * (1.0 / 3.0)) * sx * kx;
      g1 += (ay + ax * (1.0 / 3.0) + ab * (1.0 / 3.0)) * sy * ky;
      g2 += -(oy * g.hx * (1.0 / 3.0)) * sx * kx - (ox * g.hy * (1.0 / 3.0)) * sy * ky;
    }
    K[0][0] += w * amm * ia;
    K[0][1] -= w * u0 * ia;
    K[0][2] -= w * u1 * ia;
    const double gw[3] = {w * g0, w * g1, w * g2};
    for (int m = 0; m < 3; ++m) {
      K[1 + m][0] -= gw[m] * sc * ia;
      K[1 + m][1] -= gw[m] * u0 * ia;
      K[1 + m][2] -= gw[m] * u1 * ia;
    }
  }
  // B_11 restricted to the cell (face form with c+ / c- per axis, mass eps sigma_a |K|)
  const double sx2 = cxp + cxm, sy2 = cyp + cym;
  K[1][1] += ab * (1.0 / 3.0) + sx2 * g.hy + sy2 * g.hx * (1.0 / 3.0);
  K[2][2] += ab * (1.0 / 3.0) + sy2 * g.hx + sx2 * g.hy * (1.0 / 3.0);
  K[3][3] += ab * (1.0 / 9.0) + (sx2 * g.hy + sy2 * g.hx) * (1.0 / 3.0);
  K[2][3] += (cxp - cxm) * g.hy * (1.0 / 3.0);
  K[3][2] += (cxp - cxm) * g.hy * (1.0 / 3.0);
  K[1][3] += (cyp - cym) * g.hx * (1.0 / 3.0);
  K[3][1] += (cyp - cym) * g.hx * (1.0 / 3.0);
  // Gauss-Jordan inverse with partial pivoting
  double Inv[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) Inv[a][b] = a == b ? 1.0 : 0.0;
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int r = c + 1; r < 4; ++r)
      if (fabs(K[r][c]) > fabs(K[piv][c])) piv = r;
    if (piv != c)
      for (int b = 0; b < 4; ++b) {
        double t = K[c][b]; K[c][b] = K[piv][b]; K[piv][b] = t;
        t = Inv[c][b]; Inv[c][b] = Inv[piv][b]; Inv[piv][b] = t;
      }
    const double id = 1.0 / K[c][c];
    for (int b = 0; b < 4; ++b) { K[c][b] *= id; Inv[c][b] *= id; }
    for (int r = 0; r < 4; ++r) {
      if (r == c) continue;
      const double f = K[r][c];
      for (int b = 0; b < 4; ++b) { K[r][b] -= f * K[c][b]; Inv[r][b] -= f * Inv[c][b]; }
    }
  }
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) kinv[(size_t)(4 * a + b) * g.ncell + p] = Inv[a][b];
}

// ---------------------------------------------------------------- level 0 (node sublattices)
__global__ void wcell_kernel(Geo g, const double* __restrict__ sigtA, double* __restrict__ wcell) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.ncell) return;
  const double D = g.area / (3.0 * sigtA[p]);  // 1 / (3 sigma_t)
  wcell[p] = D * g.area * (0.25 / (g.hx * g.hx) + 0.25 / (g.hy * g.hy));
}

__global__ void d0_kernel(Geo g, const double* __restrict__ wcell, const double* __restrict__ absA,
                          double* __restrict__ d0) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)g.NX * g.NY) return;
  const int I = (int)(t % g.NX), J = (int)(t / g.NX);
  double s = 0.0;
  for (int dj = -1; dj <= 0; ++dj)
    for (int di = -1; di <= 0; ++di) {
      const int i = I + di, j = J + dj;
      if (i < 0 || j < 0 || i >= g.nx || j >= g.ny) continue;
      const long long p = (long long)j * g.nx + i;
      s += wcell[p] + 0.25 * absA[p];
    }
  // lumped 1/2 int_{dD} u v: a quarter of each adjacent boundary edge
  if (I == 0 || I == g.NX - 1) s += 0.25 * g.hy * ((J > 0) + (J < g.NY - 1));
  if (J == 0 || J == g.NY - 1) s += 0.25 * g.hx * ((I > 0) + (I < g.NX - 1));
  d0[t] = s;
}

// sum over the diagonal neighbours of node (I, J) of weight * u
__device__ __forceinline__ double diag_nb_sum(const Geo& g, const double* __restrict__ wcell,
                                              const double* __restrict__ u, int I, int J) {
  double s = 0.0;
  if (I < g.nx && J < g.ny) s += wcell[(long long)J * g.nx + I] * u[(long long)(J + 1) * g.NX + I + 1];
  if (I > 0 && J < g.ny) s += wcell[(long long)J * g.nx + I - 1] * u[(long long)(J + 1) * g.NX + I - 1];
  if (I < g.nx && J > 0) s += wcell[(long long)(J - 1) * g.nx + I] * u[(long long)(J - 1) * g.NX + I + 1];
  if (I > 0 && J > 0) s += wcell[(long long)(J - 1) * g.nx + I - 1] * u[(long long)(J - 1) * g.NX + I - 1];
  return s;
}

// Gauss-Seidel half sweep over the rows j with j % 2 == par (both colours at once)
__global__ void gs0_kernel(Geo g, int par, const double* __restrict__ wcell, const double* __restrict__ d0,
                           const double* __restrict__ f, double* __restrict__ u) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int rows = (g.NY - par + 1) / 2;
  if (t >= (long long)rows * g.NX) return;
  const int I = (int)(t % g.NX), J = 2 * (int)(t / g.NX) + par;
  const long long n = (long long)J * g.NX + I;
  u[n] = (f[n] + diag_nb_sum(g, wcell, u, I, J)) / d0[n];
}

// Parents of level-0 node (I, J) on level 1 (nodes (2P, 2Q), index P + mx Q): returns count
__device__ __forceinline__ int parents0(int NX, int NY, int mx, int I, int J, int* idx, double* wt) {
  int n = 0;
  const int c = (I + J) & 1;
  if (c == 0 && !(I & 1)) {
    idx[0] = (I >> 1) + mx * (J >> 1);
    wt[0] = 1.0;
    return 1;
  }
  int ci[4], cj[4], k = 0;
  if (c == 0) {  // i, j odd: the four diagonal neighbours
    for (int b = -1; b <= 1; b += 2)
      for (int a = -1; a <= 1; a += 2) { ci[k] = I + a; cj[k] = J + b; ++k; }
  } else if (I & 1) {  // i odd, j even: the two neighbours along x
    ci[0] = I - 1; cj[0] = J; ci[1] = I + 1; cj[1] = J; k = 2;
  } else {  // i even, j odd: the two neighbours along y
    ci[0] = I; cj[0] = J - 1; ci[1] = I; cj[1] = J + 1; k = 2;
  }
  for (int q = 0; q < k; ++q)
    if (ci[q] >= 0 && ci[q] < NX && cj[q] >= 0 && cj[q] < NY) idx[n++] = (ci[q] >> 1) + mx * (cj[q] >> 1);
  for (int q = 0; q < n; ++q) wt[q] = 1.0 / n;
  return n;
}

// Level-0 nodes of colour c that have level-1 node (P, Q) as a parent: up to 5
__device__ __forceinline__ int children0(int NX, int NY, int c, int P, int Q, int* ci, int* cj) {
  int k = 0;
  if (c == 0) {
    ci[k] = 2 * P; cj[k] = 2 * Q; ++k;
    for (int b = -1; b <= 1; b += 2)
      for (int a = -1; a <= 1; a += 2) { ci[k] = 2 * P + a; cj[k] = 2 * Q + b; ++k; }
  } else {
    ci[0] = 2 * P - 1; cj[0] = 2 * Q; ci[1] = 2 * P + 1; cj[1] = 2 * Q;
    ci[2] = 2 * P; cj[2] = 2 * Q - 1; ci[3] = 2 * P; cj[3] = 2 * Q + 1;
    k = 4;
  }
  int n = 0;
  for (int q = 0; q < k; ++q)
    if (ci[q] >= 0 && ci[q] < NX && cj[q] >= 0 && cj[q] < NY) { ci[n] = ci[q]; cj[n] = cj[q]; ++n; }
  return n;
}

// residual of level 0 restricted to level 1 (both colours); zeroes the level-1 iterate
__global__ void restrict0_kernel(Geo g, int mx, int my, const double* __restrict__ wcell,
                                 const double* __restrict__ d0, const double* __restrict__ f0,
                                 const double* __restrict__ u0, double* __restrict__ f1, double* __restrict__ u1) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long m = (long long)mx * my;
  const int c = blockIdx.y;
  if (t >= m) return;
  const int P = (int)(t % mx), Q = (int)(t / mx);
  int ci[5], cj[5];
  const int n = children0(g.NX, g.NY, c, P, Q, ci, cj);
  double s = 0.0;
  for (int q = 0; q < n; ++q) {
    int idx[4];
    double wt[4];
    const int np = parents0(g.NX, g.NY, mx, ci[q], cj[q], idx, wt);
    double w = 0.0;
    for (int k = 0; k < np; ++k)
      if (idx[k] == t) w = wt[k];
    const long long node = (long long)cj[q] * g.NX + ci[q];
    const double r = f0[node] - (d0[node] * u0[node] - diag_nb_sum(g, wcell, u0, ci[q], cj[q]));
    s += w * r;
  }
  f1[c * m + t] = s;
  u1[c * m + t] = 0.0;
}

__global__ void prolong0_kernel(Geo g, int mx, int my, const double* __restrict__ u1, double* __restrict__ u0) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)g.NX * g.NY) return;
  const int I = (int)(t % g.NX), J = (int)(t / g.NX);
  const int c = (I + J) & 1;
  const long long m = (long long)mx * my;
  int idx[4];
  double wt[4];
  const int np = parents0(g.NX, g.NY, mx, I, J, idx, wt);
  double e = 0.0;
  for (int k = 0; k < np; ++k) e += wt[k] * u1[c * m + idx[k]];
  u0[t] += e;
}

// Galerkin operator of level 1: A_1 = P_0^T A_0 P_0 per colour, 9-point stencil
__global__ void rap0_kernel(Geo g, int mx, int my, const double* __restrict__ wcell, const double* __restrict__ d0,
                            double* __restrict__ S1) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long m = (long long)mx * my;
  const int c = blockIdx.y;
  if (t >= m) return;
  const int P = (int)(t % mx), Q = (int)(t / mx);
  double acc[9];
  for (int k = 0; k < 9; ++k) acc[k] = 0.0;
  int ci[5], cj[5];
  const int n = children0(g.NX, g.NY, c, P, Q, ci, cj);
  for (int q = 0; q < n; ++q) {
    int idx[4];
    double wt[4];
    int np = parents0(g.NX, g.NY, mx, ci[q], cj[q], idx, wt);
    double pw = 0.0;
    for (int k = 0; k < np; ++k)
      if (idx[k] == t) pw = wt[k];
    if (pw == 0.0) continue;
    // row of A_0 at fine node (I, J): diagonal d0 and -w_K to the four diagonal neighbours
    const int I = ci[q], J = cj[q];
    for (int nb = 0; nb < 5; ++nb) {
      int I2 = I, J2 = J;
      double a;
      if (nb == 0) {
        a = d0[(long long)J * g.NX + I];
      } else {
        const int di = (nb & 1) ? 1 : -1, dj = (nb & 2) ? 1 : -1;
        I2 = I + di;
        J2 = J + dj;
        const int ic = di > 0 ? I : I - 1, jc = dj > 0 ? J : J - 1;  // the cell joining them
        if (ic < 0 || jc < 0 || ic >= g.nx || jc >= g.ny) continue;
        a = -wcell[(long long)jc * g.nx + ic];
      }
      int idx2[4];
      double wt2[4];
      const int np2 = parents0(g.NX, g.NY, mx, I2, J2, idx2, wt2);
      for (int k = 0; k < np2; ++k) {
        const int dP = idx2[k] % mx - P, dQ = idx2[k] / mx - Q;
        if (dP < -1 || dP > 1 || dQ < -1 || dQ > 1) continue;  // not reached (stencils stay 3 x 3)
        acc[(dQ + 1) * 3 + dP + 1] += pw * a * wt2[k];
      }
    }
  }
  for (int k = 0; k < 9; ++k) S1[((size_t)c * 9 + k) * m + t] = acc[k];
}

// ---------------------------------------------------------------- Cartesian levels
// bilinear parents of fine node (i, j) (fine grid mx x my) on the coarse grid of even nodes
__device__ __forceinline__ int parents9(int mx, int my, int mxc, int i, int j, int* idx, double* wt) {
  int pi[2], pj[2], ni = 0, nj = 0;
  if (!(i & 1)) pi[ni++] = i >> 1;
  else {
    pi[ni++] = (i - 1) >> 1;
    if (i + 1 < mx) pi[ni++] = (i + 1) >> 1;
  }
  if (!(j & 1)) pj[nj++] = j >> 1;
  else {
    pj[nj++] = (j - 1) >> 1;
    if (j + 1 < my) pj[nj++] = (j + 1) >> 1;
  }
  int n = 0;
  for (int b = 0; b < nj; ++b)
    for (int a = 0; a < ni; ++a) {
      idx[n] = pi[a] + mxc * pj[b];
      wt[n] = 1.0 / (ni * nj);
      ++n;
    }
  return n;
}

__device__ __forceinline__ double stencil_apply(const double* __restrict__ S, long long m, int mx, int my,
                                                const double* __restrict__ u, int i, int j, bool skip_center) {
  double s = 0.0;
  for (int dj = -1; dj <= 1; ++dj) {
    const int jj = j + dj;
    if (jj < 0 || jj >= my) continue;
    for (int di = -1; di <= 1; ++di) {
      const int ii = i + di;
      if (ii < 0 || ii >= mx || (skip_center && di == 0 && dj == 0)) continue;
      s += S[(size_t)((dj + 1) * 3 + di + 1) * m + (long long)j * mx + i] * u[(long long)jj * mx + ii];
    }
  }
  return s;
}

// four-colour Gauss-Seidel: nodes with (i % 2, j % 2) == (cg & 1, cg >> 1)
__global__ void gs9_kernel(int mx, int my, int cg, const double* __restrict__ S_all, const double* __restrict__ f_all,
                           double* __restrict__ u_all) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int ox = cg & 1, oy = cg >> 1;
  const int cx = (mx - ox + 1) / 2, cy = (my - oy + 1) / 2;
  if (t >= (long long)cx * cy) return;
  const int i = 2 * (int)(t % cx) + ox, j = 2 * (int)(t / cx) + oy;
  const long long m = (long long)mx * my;
  const int c = blockIdx.y;
  const double* S = S_all + (size_t)c * 9 * m;
  const double* f = f_all + c * m;
  double* u = u_all + c * m;
  const long long n = (long long)j * mx + i;
  u[n] = (f[n] - stencil_apply(S, m, mx, my, u, i, j, true)) / S[4 * m + n];
}

__global__ void resid9_kernel(int mx, int my, const double* __restrict__ S_all, const double* __restrict__ f_all,
                              const double* __restrict__ u_all, double* __restrict__ r_all) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long m = (long long)mx * my;
  if (t >= m) return;
  const int c = blockIdx.y;
  const int i = (int)(t % mx), j = (int)(t / mx);
  r_all[c * m + t] = f_all[c * m + t] - stencil_apply(S_all + (size_t)c * 9 * m, m, mx, my, u_all + c * m, i, j, false);
}

__global__ void restrict9_kernel(int mx, int my, int mxc, int myc, const double* __restrict__ r_all,
                                 double* __restrict__ fc_all, double* __restrict__ uc_all) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long mc = (long long)mxc * myc, m = (long long)mx * my;
  if (t >= mc) return;
  const int c = blockIdx.y;
  const int P = (int)(t % mxc), Q = (int)(t / mxc);
  double s = 0.0;
  for (int j = 2 * Q - 1; j <= 2 * Q + 1; ++j) {
    if (j < 0 || j >= my) continue;
    for (int i = 2 * P - 1; i <= 2 * P + 1; ++i) {
      if (i < 0 || i >= mx) continue;
      int idx[4];
      double wt[4];
      const int np = parents9(mx, my, mxc, i, j, idx, wt);
      for (int k = 0; k < np; ++k)
        if (idx[k] == t) s += wt[k] * r_all[c * m + (long long)j * mx + i];
    }
  }
  fc_all[c * mc + t] = s;
  uc_all[c * mc + t] = 0.0;
}

__global__ void prolong9_kernel(int mx, int my, int mxc, int myc, const double* __restrict__ uc_all,
                                double* __restrict__ u_all) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long m = (long long)mx * my, mc = (long long)mxc * myc;
  if (t >= m) return;
  const int c = blockIdx.y;
  const int i = (int)(t % mx), j = (int)(t / mx);
  int idx[4];
  double wt[4];
  const int np = parents9(mx, my, mxc, i, j, idx, wt);
  double e = 0.0;
  for (int k = 0; k < np; ++k) e += wt[k] * uc_all[c * mc + idx[k]];
  u_all[c * m + t] += e;
}

// Galerkin operator of the next level: S_c = P^T S P (both grids Cartesian)
__global__ void rap9_kernel(int mx, int my, int mxc, int myc, const double* __restrict__ S_all,
                            double* __restrict__ Sc_all) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long mc = (long long)mxc * myc, m = (long long)mx * my;
  if (t >= mc) return;
  const int c = blockIdx.y;
  const double* S = S_all + (size_t)c * 9 * m;
  const int P = (int)(t % mxc), Q = (int)(t / mxc);
  double acc[9];
  for (int k = 0; k < 9; ++k) acc[k] = 0.0;
  for (int j = 2 * Q - 1; j <= 2 * Q + 1; ++j) {
    if (j < 0 || j >= my) continue;
    for (int i = 2 * P - 1; i <= 2 * P + 1; ++i) {
      if (i < 0 || i >= mx) continue;
      int idx[4];
      double wt[4];
      int np = parents9(mx, my, mxc, i, j, idx, wt);
      double pw = 0.0;
      for (int k = 0; k < np; ++k)
        if (idx[k] == t) pw = wt[k];
      if (pw == 0.0) continue;
      const long long n = (long long)j * mx + i;
      for (int dj = -1; dj <= 1; ++dj) {
        const int j2 = j + dj;
        if (j2 < 0 || j2 >= my) continue;
        for (int di = -1; di <= 1; ++di) {
          const int i2 = i + di;
          if (i2 < 0 || i2 >= mx) continue;
          const double a = S[(size_t)((dj + 1) * 3 + di + 1) * m + n];
          if (a == 0.0) continue;
          int idx2[4];
          double wt2[4];
          const int np2 = parents9(mx, my, mxc, i2, j2, idx2, wt2);
          for (int k = 0; k < np2; ++k) {
            const int dP = idx2[k] % mxc - P, dQ = idx2[k] / mxc - Q;
            if (dP < -1 || dP > 1 || dQ < -1 || dQ > 1) continue;  // not reached (stencils stay 3 x 3)
            acc[(dQ + 1) * 3 + dP + 1] += pw * a * wt2[k];
          }
        }
      }
    }
  }
  for (int k = 0; k < 9; ++k) Sc_all[((size_t)c * 9 + k) * mc + t] = acc[k];
}

// dense inverse of the coarsest operator, one workgroup per colour (Gauss-Jordan; the
// operator is symmetric positive definite, so no pivoting)
__global__ void coarse_inverse_kernel(int mx, int my, const double* __restrict__ S_all, double* __restrict__ work_all,
                                      double* __restrict__ inv_all) {
  const int c = blockIdx.x;
  const int m = mx * my, w2 = 2 * m;
  const double* S = S_all + (size_t)c * 9 * m;
  double* W = work_all + (size_t)c * m * w2;
  double* inv = inv_all + (size_t)c * m * m;
  __shared__ double factor[kCoarseMax];
  __shared__ double piv;
  for (int e = threadIdx.x; e < m * w2; e += blockDim.x) {
    const int r = e / w2, col = e % w2;
    double v = 0.0;
    if (col < m) {
      const int dx = col % mx - r % mx, dy = col / mx - r / mx;
      if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) v = S[(size_t)((dy + 1) * 3 + dx + 1) * m + r];
    } else {
      v = (col - m == r) ? 1.0 : 0.0;
    }
    W[e] = v;
  }
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    if (threadIdx.x == 0) piv = W[(size_t)k * w2 + k];
    __syncthreads();
    for (int col = threadIdx.x; col < w2; col += blockDim.x) W[(size_t)k * w2 + col] /= piv;
    __syncthreads();
    for (int r = threadIdx.x; r < m; r += blockDim.x) factor[r] = W[(size_t)r * w2 + k];
    __syncthreads();
    for (int e = threadIdx.x; e < m * w2; e += blockDim.x) {
      const int r = e / w2, col = e % w2;
      if (r != k) W[e] -= factor[r] * W[(size_t)k * w2 + col];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) inv[e] = W[(size_t)(e / m) * w2 + m + e % m];
}

__global__ void coarse_solve_kernel(int m, const double* __restrict__ inv_all, const double* __restrict__ f_all,
                                    double* __restrict__ u_all) {
  const int c = blockIdx.x;
  const double* inv = inv_all + (size_t)c * m * m;
  for (int r = threadIdx.x; r < m; r += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += inv[(size_t)r * m + k] * f_all[c * m + k];
    u_all[c * m + r] = s;
  }
}

// ---------------------------------------------------------------- transfer to / from cells
__global__ void pc_load_kernel(Geo g, const double* __restrict__ r, const double* __restrict__ scatA,
                               double* __restrict__ f0) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)g.NX * g.NY) return;
  const int I = (int)(t % g.NX), J = (int)(t / g.NX);
  const long long nc = g.ncell;
  double s = 0.0;
  for (int dj = -1; dj <= 0; ++dj)
    for (int di = -1; di <= 0; ++di) {
      const int i = I + di, j = J + dj;
      if (i < 0 || j < 0 || i >= g.nx || j >= g.ny) continue;
      const long long p = (long long)j * g.nx + i;
      const double cx = di < 0 ? 1.0 : -1.0, cy = dj < 0 ? 1.0 : -1.0;  // the node's corner of cell p
      s += scatA[p] * r[p] - cx * r[nc + p] - cy * r[2 * nc + p] - cx * cy * r[3 * nc + p];
    }
  f0[t] = 0.25 * s;
}

__device__ __forceinline__ double cell_avg(const Geo& g, const double* __restrict__ u, int i, int j) {
  if (i < 0 || j < 0 || i >= g.nx || j >= g.ny) return 0.0;  // vacuum: zero outside the domain
  const long long n = (long long)j * g.NX + i;
  return 0.25 * (u[n] + u[n + 1] + u[n + g.NX] + u[n + g.NX + 1]);
}

// z = K_loc^{-1} r (+ Z u): out in the moment-major layout of the reduced vectors
__global__ void pc_out_kernel(Geo g, const double* __restrict__ kinv, const double* __restrict__ r,
                              const double* __restrict__ u, int rlm, double wxp, double wxm, double wyp,
                              double wym, double* __restrict__ z) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.ncell) return;
  const long long nc = g.ncell;
  const double rv[4] = {r[p], r[nc + p], r[2 * nc + p], r[3 * nc + p]};
  double out[4];
  for (int a = 0; a < 4; ++a) {
    double s = 0.0;
    for (int b = 0; b < 4; ++b) s += kinv[(size_t)(4 * a + b) * nc + p] * rv[b];
    out[a] = s;
  }
  if (u) {
    const int i = (int)(p % g.nx), j = (int)(p / g.nx);
    const long long n = (long long)j * g.NX + i;
    const double sw = u[n], se = u[n + 1], nw = u[n + g.NX], ne = u[n + g.NX + 1];
    const double avg = 0.25 * (sw + se + nw + ne);
    out[0] += avg;
    out[1] -= 0.25 * (-sw + se - nw + ne);
    out[2] -= 0.25 * (-sw - se + nw + ne);
    out[3] -= 0.25 * (sw - se - nw + ne);
    if (rlm) {
      // angular average of the reconstructed slopes of the isotropic cell averages:
      // directions with Omega_a > 0 take (avg_K - avg_up) k, the others -(avg_K - avg_down) k,
      // k = 1 in the inflow cell and 1/2 inside, zero outside the domain
      const double kxp = i == 0 ? 1.0 : 0.5, kxm = i == g.nx - 1 ? 1.0 : 0.5;
      const double kyp = j == 0 ? 1.0 : 0.5, kym = j == g.ny - 1 ? 1.0 : 0.5;
      out[1] += wxp * kxp * (avg - cell_avg(g, u, i - 1, j)) - wxm * kxm * (avg - cell_avg(g, u, i + 1, j));
      out[2] += wyp * kyp * (avg - cell_avg(g, u, i, j - 1)) - wym * kym * (avg - cell_avg(g, u, i, j + 1));
    }
  }
  for (int a = 0; a < 4; ++a) z[(size_t)a * nc + p] = out[a];
}

__global__ void pc_fill_kernel(double* __restrict__ y, long long n) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] = 0.0;
}

Geo geo_of(const lmdg_handle* h) {
  Geo g;
  g.nx = (int)h->n[0];
  g.ny = (int)h->n[1];
  g.NX = g.nx + 1;
  g.NY = g.ny + 1;
  g.ncell = h->ncell;
  g.hx = h->h[0];
  g.hy = h->h[1];
  g.area = h->area;
  return g;
}

// level l of the Cartesian hierarchy: V-cycle from level l down
void descend(lmdg_handle* h, size_t l, hipStream_t st) {
  Precond& pc = *h->pc;
  PcLevel& L = pc.lev[l];
  const long long m = (long long)L.mx * L.my;
  if (l + 1 == pc.lev.size()) {
    coarse_solve_kernel<<<2, kT, 0, st>>>((int)m, pc.cinv, L.f, L.u);
    return;
  }
  PcLevel& C = pc.lev[l + 1];
  const long long mc = (long long)C.mx * C.my;
  for (int cg = 0; cg < 4; ++cg)
    gs9_kernel<<<dim3(blocks_for((m + 3) / 4 + L.mx + L.my + 1), 2), kT, 0, st>>>(L.mx, L.my, cg, L.S, L.f, L.u);
  resid9_kernel<<<dim3(blocks_for(m), 2), kT, 0, st>>>(L.mx, L.my, L.S, L.f, L.u, L.r);
  restrict9_kernel<<<dim3(blocks_for(mc), 2), kT, 0, st>>>(L.mx, L.my, C.mx, C.my, L.r, C.f, C.u);
  descend(h, l + 1, st);
  prolong9_kernel<<<dim3(blocks_for(m), 2), kT, 0, st>>>(L.mx, L.my, C.mx, C.my, C.u, L.u);
  for (int cg = 3; cg >= 0; --cg)
    gs9_kernel<<<dim3(blocks_for((m + 3) / 4 + L.mx + L.my + 1), 2), kT, 0, st>>>(L.mx, L.my, cg, L.S, L.f, L.u);
}

void vcycle(lmdg_handle* h, hipStream_t st) {
  Precond& pc = *h->pc;
  const Geo g = geo_of(h);
  const long long nn = (long long)g.NX * g.NY;
  PcLevel& L1 = pc.lev[0];
  const long long m1 = (long long)L1.mx * L1.my;
  for (int par = 0; par < 2; ++par)
    gs0_kernel<<<blocks_for((long long)((g.NY + 1) / 2) * g.NX), kT, 0, st>>>(g, par, pc.wcell, pc.d0, pc.f0, pc.u0);
  restrict0_kernel<<<dim3(blocks_for(m1), 2), kT, 0, st>>>(g, L1.mx, L1.my, pc.wcell, pc.d0, pc.f0, pc.u0, L1.f, L1.u);
  descend(h, 0, st);
  prolong0_kernel<<<blocks_for(nn), kT, 0, st>>>(g, L1.mx, L1.my, L1.u, pc.u0);
  for (int par = 1; par >= 0; --par)
    gs0_kernel<<<blocks_for((long long)((g.NY + 1) / 2) * g.NX), kT, 0, st>>>(g, par, pc.wcell, pc.d0, pc.f0, pc.u0);
}

}  // namespace

bool pc_supported(const lmdg_handle* h, int scheme, std::string* why) {
  const char* msg = nullptr;
  if (h->dim != 2 || h->slab) msg = "the preconditioner is built for 2D handles";
  else if (scheme != LMDG_SCHEME_LMDG && scheme != LMDG_SCHEME_RLMDG) msg = "the preconditioner covers LMDG and RLMDG";
  else if (scheme == LMDG_SCHEME_RLMDG && h->recon_flags != 0)
    msg = "the preconditioner covers the two-cell reconstruction only";
  else if (h->adj_rlm) msg = "the RLMDG adjoint system is solved without the preconditioner";
  if (msg && why) *why = msg;
  return msg == nullptr;
}

size_t pc_bytes(const lmdg_handle* h) { return h->pc ? h->pc->bytes : 0; }

void pc_free(lmdg_handle* h) {
  if (!h->pc) return;
  for (void* p : h->pc->allocs)
    if (p) hipFree(p);
  delete h->pc;
  h->pc = nullptr;
}

// Build (or rebuild for new materials or another scheme) what pc_apply needs.
int pc_prepare(lmdg_handle* h, int scheme, hipStream_t st) {
  std::string why;
  if (!pc_supported(h, scheme, &why)) return set_error(h, LMDG_UNSUPPORTED, why);
  const Geo g = geo_of(h);
  if (!h->pc) {
    Precond* pc = new Precond;
    pc->NX = g.NX;
    pc->NY = g.NY;
    int mx = (g.NX + 1) / 2, my = (g.NY + 1) / 2;
    while (true) {
      PcLevel L;
      L.mx = mx;
      L.my = my;
      pc->lev.push_back(L);
      if ((long long)mx * my <= kCoarseMax) break;
      mx = (mx + 1) / 2;
      my = (my + 1) / 2;
    }
    auto alloc = [&](double** p, size_t n) {
      hipError_t e = hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(double));
      if (e != hipSuccess) return e;
      pc->allocs.push_back(*p);
      pc->bytes += std::max<size_t>(n, 1) * sizeof(double);
      return hipSuccess;
    };
    const long long nn = (long long)g.NX * g.NY;
    hipError_t e = alloc(&pc->kinv, (size_t)16 * g.ncell);
    if (e == hipSuccess) e = alloc(&pc->wcell, g.ncell);
    if (e == hipSuccess) e = alloc(&pc->d0, nn);
    if (e == hipSuccess) e = alloc(&pc->u0, nn);
    if (e == hipSuccess) e = alloc(&pc->f0, nn);
    for (PcLevel& L : pc->lev) {
      const size_t m = (size_t)L.mx * L.my;
      if (e == hipSuccess) e = alloc(&L.S, 18 * m);
      if (e == hipSuccess) e = alloc(&L.u, 2 * m);
      if (e == hipSuccess) e = alloc(&L.f, 2 * m);
      if (e == hipSuccess) e = alloc(&L.r, 2 * m);
    }
    const size_t mc = (size_t)pc->lev.back().mx * pc->lev.back().my;
    if (e == hipSuccess) e = alloc(&pc->cinv, 2 * mc * mc);
    if (e == hipSuccess) e = alloc(&pc->cwork, 4 * mc * mc);
    h->pc = pc;
    if (e != hipSuccess) {
      pc_free(h);
      return check_hip(h, e, "hipMalloc preconditioner");
    }
  }
  Precond& pc = *h->pc;
  if (pc.mg_mat != h->mat_version) {
    wcell_kernel<<<blocks_for(g.ncell), kT, 0, st>>>(g, h->d_sigtA, pc.wcell);
    d0_kernel<<<blocks_for((long long)g.NX * g.NY), kT, 0, st>>>(g, pc.wcell, h->d_absA, pc.d0);
    PcLevel& L1 = pc.lev[0];
    rap0_kernel<<<dim3(blocks_for((long long)L1.mx * L1.my), 2), kT, 0, st>>>(g, L1.mx, L1.my, pc.wcell, pc.d0, L1.S);
    for (size_t l = 0; l + 1 < pc.lev.size(); ++l) {
      PcLevel& F = pc.lev[l];
      PcLevel& C = pc.lev[l + 1];
      rap9_kernel<<<dim3(blocks_for((long long)C.mx * C.my), 2), kT, 0, st>>>(F.mx, F.my, C.mx, C.my, F.S, C.S);
    }
    PcLevel& Lc = pc.lev.back();
    coarse_inverse_kernel<<<2, kT, 0, st>>>(Lc.mx, Lc.my, Lc.S, pc.cwork, pc.cinv);
    pc.mg_mat = h->mat_version;
  }
  if (pc.kloc_mat != h->mat_version || pc.kloc_scheme != scheme) {
    kloc_kernel<<<blocks_for(g.ncell), kT, 0, st>>>(g, h->d_dirs, 4 * h->dslots, h->d_sigtA, h->d_scatA, h->d_absA,
                                                    h->cplus[0], h->cminus[0], h->cplus[1], h->cminus[1],
                                                    scheme == LMDG_SCHEME_RLMDG ? 1 : 0, pc.kinv);
    pc.kloc_mat = h->mat_version;
    pc.kloc_scheme = scheme;
  }
  return check_hip(h, hipGetLastError(), "preconditioner setup");
}

// z = M^{-1} r for every right-hand side of the handle (vectors stacked source-major).
int pc_apply(lmdg_handle* h, int scheme, const double* r, double* z, hipStream_t st) {
  int rc = pc_prepare(h, scheme, st);
  if (rc != LMDG_OK) return rc;
  Precond& pc = *h->pc;
  const Geo g = geo_of(h);
  const long long nn = (long long)g.NX * g.NY;
  const long long seg = (long long)h->np * g.ncell;
  const bool rlm = scheme == LMDG_SCHEME_RLMDG;
  // sums of the weights of the directions with Omega_x > 0, < 0, Omega_y > 0, < 0
  // (quadrant q: bit 0 set when Omega_x < 0, bit 1 when Omega_y < 0)
  const double wxp = h->qw[0] + h->qw[2], wxm = h->qw[1] + h->qw[3];
  const double wyp = h->qw[0] + h->qw[1], wym = h->qw[2] + h->qw[3];
  for (int k = 0; k < h->n_rhs; ++k) {
    const double* rk = r + k * seg;
    double* zk = z + k * seg;
    const bool two_level = h->pc_kind == LMDG_PRECOND_TWO_LEVEL;
    if (two_level) {
      pc_load_kernel<<<blocks_for(nn), kT, 0, st>>>(g, rk, h->d_scatA, pc.f0);
      pc_fill_kernel<<<blocks_for(nn), kT, 0, st>>>(pc.u0, nn);
      for (int c = 0; c < h->pc_cycles; ++c) vcycle(h, st);
    }
    pc_out_kernel<<<blocks_for(g.ncell), kT, 0, st>>>(g, pc.kinv, rk, two_level ? pc.u0 : nullptr, rlm ? 1 : 0, wxp,
                                                      wxm, wyp, wym, zk);
  }
  return check_hip(h, hipGetLastError(), "preconditioner");
}

}  // namespace lmdg
