// Reductions into moment vectors and the B_11 stencil on a uniform 3D mesh.
//
// Moments of the trilinear Legendre basis, index m = bx + 2 by + 4 bz: 1, xi, eta,
// xi eta, zeta, xi zeta, eta zeta, xi eta zeta.  Slope moments are m = 1..7.
#include "internal.h"

#include <type_traits>

namespace lmdg {
namespace {

constexpr int kBlock3 = 256;

inline int grid3(long long n) {
  long long g = (n + kBlock3 - 1) / kBlock3;
  return (int)std::min<long long>(std::max<long long>(g, 1), 4096);
}

struct Geo3 {
  int n[3];
  double A[3];        // face measures h_y h_z, h_x h_z, h_x h_y
  double cp[3], cm[3];  // sum over directions with Omega_a > 0 of w Omega_a, and with Omega_a < 0 of w |Omega_a|
  long long stride[3];
};

struct OctMoments {
  double w[8], a[8][3];  // per octant: sum w, sum w |Omega_a|
};

__device__ __forceinline__ double third_pow(int m) {
  const int k = (m & 1) + ((m >> 1) & 1) + ((m >> 2) & 1);
  return k == 0 ? 1.0 : (k == 1 ? 1.0 / 3.0 : (k == 2 ? 1.0 / 9.0 : 1.0 / 27.0));
}

// B_11 X_1 on one cell (Sec. 3.2, eq-lmdg-psi1) in the face form of App. C: isotropic
// slopes make the streaming volume term vanish (condition (ii)); on a face with normal
// +e_a between K- and K+ the directions with Omega_a > 0 take K-'s trace, the others
// K+'s, giving int_F (c+ u_- - c- u_+)(v_- - v_+) with exterior traces zero.  The trace
// of u at xi_a = +-1 has tangential coefficients u[t] +- u[t | e_a] for the tangential
// modes t (u[0] = 0: only slopes), and the face mass of mode t is A_a (1/3)^{#bits t}.
// Mass term: eps sigma_a V (1/3)^{#bits m} u[m].
// xs(m, a, side): slope moment m of the cell displaced by side (-1, 0, +1) along axis a;
// called only for cells inside the mesh.
template <typename XS>
__device__ __forceinline__ void b11_cell3_acc(XS xs, const Geo3& g, const int idx[3], double absA, double y[8]) {
#pragma unroll
  for (int m = 1; m < 8; ++m) y[m] = absA * third_pow(m) * xs(m, 0, 0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int nb = 1 << a;
    const double A = g.A[a], cp = g.cp[a], cm = g.cm[a];
    const bool has_hi = idx[a] + 1 < g.n[a], has_lo = idx[a] > 0;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      if (t & nb) continue;
      const double fm = A * third_pow(t);
      const double xt = t ? xs(t, 0, 0) : 0.0, xn = xs(t | nb, 0, 0);
      {  // face at xi_a = +1: this cell is K-
        const double un = has_hi ? (t ? xs(t, a, 1) : 0.0) - xs(t | nb, a, 1) : 0.0;
        const double J = cp * (xt + xn) - cm * un;
        if (t) y[t] += fm * J;
        y[t | nb] += fm * J;
      }
      {  // face at xi_a = -1: this cell is K+
        const double un = has_lo ? (t ? xs(t, a, -1) : 0.0) + xs(t | nb, a, -1) : 0.0;
        const double J = cp * un - cm * (xt - xn);
        if (t) y[t] -= fm * J;
        y[t | nb] += fm * J;
      }
    }
    // one axis at a time: keeps the neighbour loads of the three axes from being hoisted
    // together (register pressure of the fully unrolled form)
    __builtin_amdgcn_sched_barrier(0);
  }
}
__device__ __forceinline__ void b11_cell3(const double* x, long long nc, const Geo3& g, const int idx[3], long long p,
                                          double absA, double y[8]) {
  b11_cell3_acc([&](int m, int a, int side) { return x[m * nc + p + side * g.stride[a]]; }, g, idx, absA, y);
}

// G Sigma_0^T x_0 on one cell: the second block row applied to x_0 copied to every
// direction, summed per octant through sum w and sum w |Omega_a| (the rows of the 3D
// sweep kernel evaluated with psi = x_0; upwind slopes k (u - u_up), k = 1 in the
// inflow cell of a line, traces zero outside the mesh).  Rows indexed by moment.
// The values of x_0 it reads, at p + d for the 25 offsets with |d|_1 <= 2, are loaded
// once into registers (zero outside the mesh); the octant loop is unrolled, so every
// access below has a constant index (nb_index).
__host__ __device__ constexpr int nb_index(int dx, int dy, int dz) {
  // 0: the cell; 1..6: +-e_a; 7..12: +-2 e_a; 13..24: +-e_a +-e_b (a < b)
  return (dx == 0 && dy == 0 && dz == 0) ? 0
         : (dy == 0 && dz == 0) ? ((dx == 1 || dx == -1) ? 1 + (dx < 0) : 7 + (dx < 0))
         : (dx == 0 && dz == 0) ? ((dy == 1 || dy == -1) ? 3 + (dy < 0) : 9 + (dy < 0))
         : (dx == 0 && dy == 0) ? ((dz == 1 || dz == -1) ? 5 + (dz < 0) : 11 + (dz < 0))
         : (dz == 0) ? 13 + 2 * (dx < 0) + (dy < 0)
         : (dy == 0) ? 17 + 2 * (dx < 0) + (dz < 0)
                     : 21 + 2 * (dy < 0) + (dz < 0);
}

// x0at(dx, dy, dz): x_0 of the cell at offset (dx, dy, dz), called only inside the mesh.
template <bool RLM, typename X0>
__device__ __forceinline__ void iso_g3_acc(X0 x0at, const Geo3& g, const int idx[3], double absA,
                                           const OctMoments& om, double out[8]) {
  constexpr int NNB = RLM ? 25 : 7;
  double nb[NNB];
#pragma unroll
  for (int dz = -2; dz <= 2; ++dz)
#pragma unroll
    for (int dy = -2; dy <= 2; ++dy)
#pragma unroll
      for (int dx = -2; dx <= 2; ++dx) {
        const int l1 = (dx < 0 ? -dx : dx) + (dy < 0 ? -dy : dy) + (dz < 0 ? -dz : dz);
        if (l1 > (RLM ? 2 : 1)) continue;
        double v = 0.0;
        const int ii = idx[0] + dx, jj = idx[1] + dy, kk = idx[2] + dz;
        if (ii >= 0 && ii < g.n[0] && jj >= 0 && jj < g.n[1] && kk >= 0 && kk < g.n[2])
          v = x0at(dx, dy, dz);
        nb[nb_index(dx, dy, dz)] = v;
      }
#pragma unroll
  for (int m = 0; m < 8; ++m) out[m] = 0.0;
  const double v = nb[0];
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    int s[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) s[a] = ((o >> a) & 1) ? -1 : 1;
    // value at the cell displaced by -s_a along the axes in `mask` (twice along mult_a)
    auto val = [&](int mask, int mult_a) -> double {
      int d[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) d[a] = ((mask >> a) & 1) ? -s[a] * (a == mult_a ? 2 : 1) : 0;
      return nb[nb_index(d[0], d[1], d[2])];
    };
    const double W = om.w[o];
    double kap[3], up[3], c[3];
    bool has_up[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      has_up[a] = s[a] > 0 ? idx[a] > 0 : idx[a] < g.n[a] - 1;
      kap[a] = has_up[a] ? 0.5 : 1.0;
      up[a] = val(1 << a, -1);
      c[a] = s[a] * kap[a] * (v - up[a]);
    }
    if (!RLM) {
#pragma unroll
      for (int a = 0; a < 3; ++a) out[1 << a] += s[a] * g.A[a] * om.a[o][a] * (up[a] - v);
      continue;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int nba = 1 << a;
      // outflow face value of the upwind cell along a
      double T = 0.0;
      if (has_up[a]) {
        const bool up_first = s[a] > 0 ? idx[a] - 1 == 0 : idx[a] + 1 == g.n[a] - 1;
        T = up[a] + (up_first ? 1.0 : 0.5) * (up[a] - val(nba, a));
      }
      // slope mass term: sigma_t V / 3 of L_11 R minus (sigma_s/eps) V / 3 of M_1 P_1 R
      double row = s[a] * g.A[a] * om.a[o][a] * (T - v) + g.A[a] * om.a[o][a] * c[a] + absA / 3.0 * W * c[a];
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if (b == a) continue;
        // a-slope of the b-upwind cell (it shares K's index along a, so the same k_a)
        const double cab = has_up[b] ? s[a] * kap[a] * (up[b] - val((1 << b) | nba, -1)) : 0.0;
        row += g.A[b] * om.a[o][b] * (c[a] - cab) / 3.0;
      }
      out[nba] += row;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = a + 1; b < 3; ++b) {
        const double cba = has_up[a] ? s[b] * kap[b] * (up[a] - val((1 << a) | (1 << b), -1)) : 0.0;  // b-slope of Ua
        const double cab = has_up[b] ? s[a] * kap[a] * (up[b] - val((1 << a) | (1 << b), -1)) : 0.0;  // a-slope of Ub
        out[(1 << a) | (1 << b)] += (s[a] * g.A[a] * om.a[o][a] * (cba - c[b]) +
                                     s[b] * g.A[b] * om.a[o][b] * (cab - c[a])) / 3.0;
      }
    // one octant at a time (register pressure)
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Right-hand side and recovery from the per-octant sweep sums (3D analogue of
// combine_lm_kernel; K x is apply3_tiled_kernel below).  Sweep outputs s: [P_0, xi, eta,
// zeta rows (, xi eta, xi zeta, eta zeta rows, P_1 R xi, eta, zeta)].
template <typename R, bool RLM, int MODE>
__global__ void __launch_bounds__(kBlock3) combine3_kernel(int nr, long long nc, const double* __restrict__ x_all,
                                                          const R* __restrict__ part_all, double* __restrict__ out_all) {
  static_assert(MODE == kRhs || MODE == kRecover, "K x is apply3_tiled_kernel");
  constexpr int NOUT = RLM ? 10 : 4;
  for (long long pr = blockIdx.x * (long long)blockDim.x + threadIdx.x; pr < nr * nc;
       pr += (long long)gridDim.x * blockDim.x) {
    const long long rh = pr / nc, p = pr - rh * nc;
    const R* part = part_all + rh * 8 * NOUT * nc;
    double* out = out_all + rh * 8 * nc;
    // rows the mode reads: P_0 and the slope rows for the right-hand side, P_0 and the
    // P_1 R rows for the recovery (RLMDG sweeps produce the P_1 R rows only for the latter)
    double s[NOUT];
#pragma unroll
    for (int m = 0; m < NOUT; ++m) {
      double acc = 0;
      const bool used = !RLM || (MODE == kRecover ? (m == 0 || m >= 7) : m < 7);
      if (used) {
#pragma unroll
        for (int o = 0; o < 8; ++o) acc += (double)part[((long long)o * NOUT + m) * nc + p];
      }
      s[m] = acc;
    }
    out[p] = s[0];
    if constexpr (MODE == kRhs) {
      // the sweep's slope rows already hold G Psi (Sigma M_1 P_1 R taken per direction)
      out[1 * nc + p] = s[1];
      out[2 * nc + p] = s[2];
      out[4 * nc + p] = s[3];
      out[3 * nc + p] = RLM ? s[4] : 0.0;
      out[5 * nc + p] = RLM ? s[5] : 0.0;
      out[6 * nc + p] = RLM ? s[6] : 0.0;
      out[7 * nc + p] = 0.0;
    } else {  // recovery: Phi_1 = -X_1 + P_1 R Psi_0
      const double* x = x_all + rh * 8 * nc;
      for (int m = 1; m < 8; ++m) {
        double v = -x[m * nc + p];
        if (RLM && (m == 1 || m == 2 || m == 4)) v += s[m == 1 ? 7 : (m == 2 ? 8 : 9)];
        out[m * nc + p] = v;
      }
    }
  }
}

// K x (modes kApply and kApplyDefect) with the x stencils read from LDS.  A workgroup
// owns a tile of kTX x kTY columns (one cell per thread and plane) and marches through
// kZC planes of one right-hand side.  Per plane k it stages x_0 of planes k - 1, k, k + 1
// with a halo of two cells in x and y (a ring of three planes) and the slope moments of
// plane k with a halo of one; each thread keeps its own column's x_0 at k +- 2 and slopes
// at k +- 1 in registers.  b11_cell3_acc and iso_g3_acc read the staged values through
// accessors; the octant partials are streamed as in combine3_kernel.
constexpr int kTX = 64, kTY = 4, kZC = 16;
template <typename R, bool RLM, int MODE>
__global__ void __launch_bounds__(kTX * kTY) apply3_tiled_kernel(int nr, Geo3 g, OctMoments om,
                                                                 const double* __restrict__ x_all,
                                                                 const R* __restrict__ part_all,
                                                                 const double* __restrict__ absA,
                                                                 double* __restrict__ out_all) {
  constexpr int NOUT = RLM ? 10 : 4;
  constexpr int H = 2;                                 // x_0 halo
  constexpr int PX = kTX + 2 * H, PY = kTY + 2 * H;    // x_0 plane tile
  constexpr int SX = kTX + 2, SY = kTY + 2;            // slope plane tile
  constexpr int NT = kTX * kTY;
  __shared__ double x0s[3][PY][PX];
  __shared__ double sls[7][SY][SX];
  // the octant moments are read from LDS inside the plane loop: its barriers keep the
  // compiler from hoisting the per-octant products out of the loop into registers
  __shared__ OctMoments oms;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const long long nxy = (long long)nx * ny, nc = nxy * nz;
  const int ntx = (nx + kTX - 1) / kTX, nty = (ny + kTY - 1) / kTY, ntz = (nz + kZC - 1) / kZC;
  // tiles in (x, y, z chunk, right-hand side) order.  Workgroups are dispatched to the
  // eight XCDs in turn and each XCD has its own L2: consecutive tiles (which share
  // halos) go to one XCD
  const int G = gridDim.x, b = blockIdx.x;
  const int lb = (G & 7) ? b : (b & 7) * (G >> 3) + (b >> 3);
  if (lb >= ntx * nty * ntz * nr) return;
  int rest = lb;
  const int bx = rest % ntx;
  rest /= ntx;
  const int by = rest % nty;
  rest /= nty;
  const int bz = rest % ntz;
  const int rh = rest / ntz;
  const int tid = threadIdx.x, tx = tid % kTX, ty = tid / kTX;
  const int i0 = bx * kTX, j0 = by * kTY, k0 = bz * kZC, k1 = min(nz, k0 + kZC);
  const int i = i0 + tx, j = j0 + ty;
  const bool act = i < nx && j < ny;
  const double* x = x_all + (long long)rh * 8 * nc;
  const R* part = part_all + (long long)rh * 8 * NOUT * nc;
  double* out = out_all + (long long)rh * 8 * nc;
  const long long col = (long long)j * nx + i;  // own column (valid where act)

  // x_0 of plane kk (zeros outside the mesh) into ring slot kk mod 3
  auto stage_x0 = [&](int kk) {
    double(*dst)[PX] = x0s[(kk + 3) % 3];
    for (int e = tid; e < PY * PX; e += NT) {
      const int hy = e / PX, hx = e - hy * PX;
      const int ii = i0 - H + hx, jj = j0 - H + hy;
      double v = 0.0;
      if (kk >= 0 && kk < nz && ii >= 0 && ii < nx && jj >= 0 && jj < ny) v = x[kk * nxy + (long long)jj * nx + ii];
      dst[hy][hx] = v;
    }
  };
  auto stage_slopes = [&](int kk) {
    for (int e = tid; e < 7 * SY * SX; e += NT) {
      const int m = e / (SY * SX), r2 = e - m * (SY * SX);
      const int hy = r2 / SX, hx = r2 - hy * SX;
      const int ii = i0 - 1 + hx, jj = j0 - 1 + hy;
      double v = 0.0;
      if (ii >= 0 && ii < nx && jj >= 0 && jj < ny) v = x[(m + 1) * nc + kk * nxy + (long long)jj * nx + ii];
      sls[m][hy][hx] = v;
    }
  };
  if (tid < 8) {
    oms.w[tid] = om.w[tid];
#pragma unroll
    for (int a = 0; a < 3; ++a) oms.a[tid][a] = om.a[tid][a];
  }
  double x0m2 = 0.0, x0p2 = 0.0, slm1[7], slp1[7];
#pragma unroll
  for (int m = 0; m < 7; ++m) slm1[m] = slp1[m] = 0.0;
  if (act && k0 >= 2) x0m2 = x[(k0 - 2) * nxy + col];
  if (act && k0 >= 1) {
#pragma unroll
    for (int m = 0; m < 7; ++m) slm1[m] = x[(m + 1) * nc + (k0 - 1) * nxy + col];
  }
  stage_x0(k0 - 1);
  stage_x0(k0);
  for (int k = k0; k < k1; ++k) {
    const long long p = k * nxy + col;
    // octant sums of the rows K x reads (the loads stay in flight through the staging)
    double sv[7];
#pragma unroll
    for (int m = 0; m < 7; ++m) {
      double acc = 0;
      if (act && (RLM || m < 4)) {
#pragma unroll
        for (int o = 0; o < 8; ++o) acc += (double)part[((long long)o * NOUT + m) * nc + p];
      }
      sv[m] = acc;
    }
    stage_x0(k + 1);
    stage_slopes(k);
    x0p2 = (act && k + 2 < nz) ? x[(k + 2) * nxy + col] : 0.0;
#pragma unroll
    for (int m = 0; m < 7; ++m) slp1[m] = (act && k + 1 < nz) ? x[(m + 1) * nc + (k + 1) * nxy + col] : 0.0;
    __syncthreads();
    if (act) {
      const int idx[3] = {i, j, k};
      const int c0 = (k + 3) % 3, cm1 = (k + 2) % 3, cp1 = (k + 4) % 3;
      auto xs = [&](int m, int a, int side) -> double {
        if (a == 2 && side != 0) return side > 0 ? slp1[m - 1] : slm1[m - 1];
        const int dx = a == 0 ? side : 0, dy = a == 1 ? side : 0;
        return sls[m - 1][ty + 1 + dy][tx + 1 + dx];
      };
      auto x0at = [&](int dx, int dy, int dz) -> double {
        if (dz == 2) return x0p2;
        if (dz == -2) return x0m2;
        const int sl = dz == 0 ? c0 : (dz > 0 ? cp1 : cm1);
        return x0s[sl][ty + H + dy][tx + H + dx];
      };
      double y[8];
      b11_cell3_acc(xs, g, idx, absA[p], y);
      double gr[8];
      gr[0] = 0.0;
      gr[1] = sv[1];
      gr[2] = sv[2];
      gr[4] = sv[3];
      gr[3] = RLM ? sv[4] : 0.0;
      gr[5] = RLM ? sv[5] : 0.0;
      gr[6] = RLM ? sv[6] : 0.0;
      gr[7] = 0.0;
      if constexpr (MODE == kApply) {
        out[p] = x0at(0, 0, 0) - sv[0];
#pragma unroll
        for (int m = 1; m < 8; ++m) out[m * nc + p] = y[m] - gr[m];
      } else {
        double gi[8];
        iso_g3_acc<RLM>(x0at, g, idx, absA[p], oms, gi);
        out[p] = sv[0];
#pragma unroll
        for (int m = 1; m < 8; ++m) out[m * nc + p] = y[m] - gi[m] + gr[m];
      }
      // registers for the next plane: x_0 at k - 1 and the slopes at k
      x0m2 = x0s[cm1][ty + H][tx + H];
#pragma unroll
      for (int m = 0; m < 7; ++m) slm1[m] = sls[m][ty + 1][tx + 1];
    }
    __syncthreads();
  }
}

// Sweep outputs in the ABI layout: LMDG 8 rows [P_0 ; Sigma L_10 rows by moment],
// RLMDG 11 rows [P_0 ; Sigma (L_10 + L_11 R) rows by moment ; P_1 R xi, eta, zeta].
template <typename R, bool RLM>
__global__ void sum_octants_kernel(int nr, long long nc, const R* __restrict__ part_all, double* __restrict__ out_all) {
  constexpr int NOUT = RLM ? 10 : 4;
  constexpr int NABI = RLM ? 11 : 8;
  // internal output feeding each ABI row (-1: zero)
  constexpr int map_l[8] = {0, 1, 2, -1, 3, -1, -1, -1};
  constexpr int map_r[11] = {0, 1, 2, 4, 3, 5, 6, -1, 7, 8, 9};
  for (long long pr = blockIdx.x * (long long)blockDim.x + threadIdx.x; pr < nr * nc;
       pr += (long long)gridDim.x * blockDim.x) {
    const long long rh = pr / nc, p = pr - rh * nc;
    const R* part = part_all + rh * 8 * NOUT * nc;
    double* out = out_all + rh * NABI * nc;
    for (int row = 0; row < NABI; ++row) {
      const int m = RLM ? map_r[row] : map_l[row];
      double acc = 0;
      if (m >= 0)
        for (int o = 0; o < 8; ++o) acc += (double)part[((long long)o * NOUT + m) * nc + p];
      out[row * nc + p] = acc;
    }
  }
}

Geo3 geo3(const lmdg_handle* h) {
  Geo3 g;
  for (int a = 0; a < 3; ++a) {
    g.n[a] = (int)h->n[a];
    g.cp[a] = h->cplus[a];
    g.cm[a] = h->cminus[a];
  }
  g.A[0] = h->h[1] * h->h[2];
  g.A[1] = h->h[0] * h->h[2];
  g.A[2] = h->h[0] * h->h[1];
  g.stride[0] = 1;
  g.stride[1] = g.n[0];
  g.stride[2] = (long long)g.n[0] * g.n[1];
  return g;
}

__global__ void b11_apply3_kernel(Geo3 g, const double* __restrict__ x, const double* __restrict__ absA,
                                  double* __restrict__ y) {
  const long long nc = (long long)g.n[0] * g.n[1] * g.n[2];
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < nc;
       p += (long long)gridDim.x * blockDim.x) {
    const int idx[3] = {(int)(p % g.n[0]), (int)((p / g.n[0]) % g.n[1]), (int)(p / ((long long)g.n[0] * g.n[1]))};
    double v[8];
    b11_cell3(x, nc, g, idx, p, absA[p], v);
    y[p] = 0.0;
    for (int m = 1; m < 8; ++m) y[m * nc + p] = v[m];
  }
}

}  // namespace

void launch_combine3(lmdg_handle* h, int scheme, int prec, int mode, const double* x, double* out, hipStream_t st) {
  const Geo3 g = geo3(h);
  OctMoments om;
  for (int o = 0; o < 8; ++o) {
    om.w[o] = h->qw[o];
    om.a[o][0] = h->qax[o];
    om.a[o][1] = h->qay[o];
    om.a[o][2] = h->qaz[o];
  }
  const int nr = h->n_rhs;
  const int grid = grid3(h->ncell * nr);
  const long long tiles = (long long)((g.n[0] + kTX - 1) / kTX) * ((g.n[1] + kTY - 1) / kTY) *
                          ((g.n[2] + kZC - 1) / kZC) * nr;
  const int grid_t = (int)(tiles < 8 ? tiles : (tiles + 7) / 8 * 8);
  const bool rlm = scheme == LMDG_SCHEME_RLMDG;
  auto go = [&](auto r_tag, auto rlm_tag) {
    using R = decltype(r_tag);
    constexpr bool RLM = decltype(rlm_tag)::value;
    const R* part = (const R*)h->ws.part;
    switch (mode) {
      case kApply:
        hipLaunchKernelGGL((apply3_tiled_kernel<R, RLM, kApply>), dim3(grid_t), dim3(kTX * kTY), 0, st, nr, g, om, x,
                           part, h->d_absA, out);
        break;
      case kApplyDefect:
        hipLaunchKernelGGL((apply3_tiled_kernel<R, RLM, kApplyDefect>), dim3(grid_t), dim3(kTX * kTY), 0, st, nr, g,
                           om, x, part, h->d_absA, out);
        break;
      case kRhs:
        hipLaunchKernelGGL((combine3_kernel<R, RLM, kRhs>), dim3(grid), dim3(kBlock3), 0, st, nr, h->ncell, x, part,
                           out);
        break;
      default:
        hipLaunchKernelGGL((combine3_kernel<R, RLM, kRecover>), dim3(grid), dim3(kBlock3), 0, st, nr, h->ncell, x,
                           part, out);
    }
  };
  if (prec == LMDG_PREC_FP64) {
    if (rlm) go(double(), std::true_type()); else go(double(), std::false_type());
  } else {
    if (rlm) go(float(), std::true_type()); else go(float(), std::false_type());
  }
}

void launch_sum_octants(lmdg_handle* h, int scheme, int prec, double* out, hipStream_t st) {
  const int nr = h->n_rhs;
  const int grid = grid3(h->ncell * nr);
  const bool rlm = scheme == LMDG_SCHEME_RLMDG;
  if (prec == LMDG_PREC_FP64) {
    if (rlm)
      hipLaunchKernelGGL((sum_octants_kernel<double, true>), dim3(grid), dim3(kBlock3), 0, st, nr, h->ncell,
                         (const double*)h->ws.part, out);
    else
      hipLaunchKernelGGL((sum_octants_kernel<double, false>), dim3(grid), dim3(kBlock3), 0, st, nr, h->ncell,
                         (const double*)h->ws.part, out);
  } else {
    if (rlm)
      hipLaunchKernelGGL((sum_octants_kernel<float, true>), dim3(grid), dim3(kBlock3), 0, st, nr, h->ncell,
                         (const float*)h->ws.part, out);
    else
      hipLaunchKernelGGL((sum_octants_kernel<float, false>), dim3(grid), dim3(kBlock3), 0, st, nr, h->ncell,
                         (const float*)h->ws.part, out);
  }
}

void launch_b11_3d(lmdg_handle* h, const double* x, double* y, hipStream_t st) {
  hipLaunchKernelGGL(b11_apply3_kernel, dim3(grid3(h->ncell)), dim3(kBlock3), 0, st, geo3(h), x, h->d_absA, y);
}

}  // namespace lmdg
