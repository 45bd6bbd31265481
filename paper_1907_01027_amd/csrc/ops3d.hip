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
__device__ __forceinline__ void b11_cell3(const double* x, long long nc, const Geo3& g, const int idx[3], long long p,
                                          double absA, double y[8]) {
#pragma unroll
  for (int m = 1; m < 8; ++m) y[m] = absA * third_pow(m) * x[m * nc + p];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int nb = 1 << a;
    const double A = g.A[a], cp = g.cp[a], cm = g.cm[a];
    const bool has_hi = idx[a] + 1 < g.n[a], has_lo = idx[a] > 0;
    const long long ph = p + g.stride[a], pl = p - g.stride[a];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      if (t & nb) continue;
      const double fm = A * third_pow(t);
      const double xt = t ? x[t * nc + p] : 0.0, xn = x[(t | nb) * nc + p];
      {  // face at xi_a = +1: this cell is K-
        const double un = has_hi ? (t ? x[t * nc + ph] : 0.0) - x[(t | nb) * nc + ph] : 0.0;
        const double J = cp * (xt + xn) - cm * un;
        if (t) y[t] += fm * J;
        y[t | nb] += fm * J;
      }
      {  // face at xi_a = -1: this cell is K+
        const double un = has_lo ? (t ? x[t * nc + pl] : 0.0) + x[(t | nb) * nc + pl] : 0.0;
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

template <bool RLM>
__device__ __forceinline__ void iso_g3(const double* __restrict__ x0, const Geo3& g, const int idx[3], long long p,
                                       double absA, const OctMoments& om, double out[8]) {
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
          v = x0[p + dx * g.stride[0] + dy * g.stride[1] + dz * g.stride[2]];
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
  }
}

// K x, right-hand side and recovery from the per-octant sweep sums (3D analogue of
// combine_lm_kernel).  Sweep outputs s: [P_0, xi, eta, zeta rows (, xi eta, xi zeta,
// eta zeta rows, P_1 R xi, eta, zeta)].
template <typename R, bool RLM, int MODE>
__global__ void __launch_bounds__(kBlock3) combine3_kernel(int nr, Geo3 g, OctMoments om, const double* __restrict__ x_all,
                                const R* __restrict__ part_all, const double* __restrict__ absA,
                                double* __restrict__ out_all) {
  constexpr int NOUT = RLM ? 10 : 4;
  const long long nc = (long long)g.n[0] * g.n[1] * g.n[2];
  for (long long pr = blockIdx.x * (long long)blockDim.x + threadIdx.x; pr < nr * nc;
       pr += (long long)gridDim.x * blockDim.x) {
    const long long rh = pr / nc, p = pr - rh * nc;
    const double* x = x_all ? x_all + rh * 8 * nc : nullptr;
    const R* part = part_all + rh * 8 * NOUT * nc;
    double* out = out_all + rh * 8 * nc;
    // rows the mode reads: operator rows (P_0 and the slope rows) for K x and the
    // right-hand side, P_0 and the P_1 R rows for the recovery (RLMDG sweeps produce
    // the P_1 R rows only for the latter)
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
    // the sweep's slope rows already hold G Psi (Sigma M_1 P_1 R taken per direction)
    double gr[8];
    gr[0] = 0.0;
    gr[1] = s[1];
    gr[2] = s[2];
    gr[4] = s[3];
    gr[3] = RLM ? s[4] : 0.0;
    gr[5] = RLM ? s[5] : 0.0;
    gr[6] = RLM ? s[6] : 0.0;
    gr[7] = 0.0;
    const int idx[3] = {(int)(p % g.n[0]), (int)((p / g.n[0]) % g.n[1]), (int)(p / ((long long)g.n[0] * g.n[1]))};
    if constexpr (MODE == kApply || MODE == kApplyDefect) {
      double y[8], gi[8];
      __builtin_amdgcn_sched_barrier(0);
      b11_cell3(x, nc, g, idx, p, absA[p], y);
      if constexpr (MODE == kApply) {
        out[p] = x[p] - s[0];
#pragma unroll
        for (int m = 1; m < 8; ++m) out[m * nc + p] = y[m] - gr[m];
      } else {
        iso_g3<RLM>(x, g, idx, p, absA[p], om, gi);
        out[p] = s[0];
#pragma unroll
        for (int m = 1; m < 8; ++m) out[m * nc + p] = y[m] - gi[m] + gr[m];
      }
    } else if constexpr (MODE == kRhs) {
      out[p] = s[0];
      for (int m = 1; m < 8; ++m) out[m * nc + p] = gr[m];
    } else {  // recovery: Phi_1 = -X_1 + P_1 R Psi_0
      out[p] = s[0];
      for (int m = 1; m < 8; ++m) {
        double v = -x[m * nc + p];
        if (RLM && (m == 1 || m == 2 || m == 4)) v += s[m == 1 ? 7 : (m == 2 ? 8 : 9)];
        out[m * nc + p] = v;
      }
    }
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
  const bool rlm = scheme == LMDG_SCHEME_RLMDG;
  auto go = [&](auto r_tag, auto rlm_tag) {
    using R = decltype(r_tag);
    constexpr bool RLM = decltype(rlm_tag)::value;
    const R* part = (const R*)h->ws.part;
    switch (mode) {
      case kApply:
        hipLaunchKernelGGL((combine3_kernel<R, RLM, kApply>), dim3(grid), dim3(kBlock3), 0, st, nr, g, om, x, part,
                           h->d_absA, out);
        break;
      case kApplyDefect:
        hipLaunchKernelGGL((combine3_kernel<R, RLM, kApplyDefect>), dim3(grid), dim3(kBlock3), 0, st, nr, g, om, x,
                           part, h->d_absA, out);
        break;
      case kRhs:
        hipLaunchKernelGGL((combine3_kernel<R, RLM, kRhs>), dim3(grid), dim3(kBlock3), 0, st, nr, g, om, x, part,
                           h->d_absA, out);
        break;
      default:
        hipLaunchKernelGGL((combine3_kernel<R, RLM, kRecover>), dim3(grid), dim3(kBlock3), 0, st, nr, g, om, x, part,
                           h->d_absA, out);
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
