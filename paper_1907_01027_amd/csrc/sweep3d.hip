// Transport sweeps on a uniform 3D Cartesian mesh (gfx950): the standard Q^1 scheme
// (eq-Ljk with trilinear elements) and the low-memory schemes LMDG and RLMDG.
//
// Work decomposition.  A work item is (octant o, strip s of 16 rows along y, block b of
// CB columns along x, right-hand side).  It carries its 16 x CB column of cells through
// every plane along z in sweep order, so that the z-inflow of a cell is the z-outflow the
// same lane produced one plane earlier and never leaves the registers.  The workgroup
// holds every direction slot of the octant: lanes are 16 rows x 4 slots per wave, W waves.
// Inside an item the cells are visited in skewed order: at step tau, row r handles the
// cell with index lambda = tau - r in the sequence (plane, column) of the block, lambda =
// plane * CB + column.  Then
//   x-inflow  the lane's previous cell (registers), or in the block's first column the
//             x-outflow of block b - 1 at the same plane and row (x-edge buffer);
//   y-inflow  the lane of the row below, whose previous step handled the same cell (DPP
//             row shift); row 0 takes the y-outflow of strip s - 1 (y-edge buffer);
//   z-inflow  the lane's own outflow CB steps earlier: the steps are unrolled in periods
//             of CB, and step u of a period reads and rewrites register slot u.
// Row r trails row 0 by r steps, so in period p the rows cover planes p - L .. p with
// L = ceil(15 / CB); plane q is complete after period q + L.  Per period the item stages
// the coefficients of plane p + 1 in LDS (a ring of L + 2 plane buffers whose slot for a
// cell is its sequence index lambda modulo (L + 2) CB: one add and a mask per step where
// that is a power of two, an add, compare and select otherwise), sums its outputs
// over the slots and waves of the octant, and publishes how many periods it has completed.
// Before period p it waits for (s - 1, b) to have completed period p + L (row 15 of the
// strip below has then passed every cell of plane p that row 0 handles in period p) and
// for (s, b - 1) to have completed period p + 1 only: the x traces a row takes in period
// p, the last column of plane p - (r >> log2 CB), leave block b - 1 by its period p + 1
// for every row r.
//
// Exchange through global memory uses agent-scope atomic loads and stores only (edge
// traces and progress words), so no cache maintenance is needed: a wave waits for its own
// trace stores to complete before the workgroup barrier that precedes the progress store,
// and a consumer issues its trace loads after the barrier that follows its wait.
//
// Local solves.  LMDG and RLMDG follow Sec. 3.2 (L_00, scalar per cell and direction) and
// Sec. 3.3 (L~_00 = L_00 + L_01 R with the upwind slopes c_a = s_a k_a (psi - psi_up,a),
// k_a = 1 in the inflow cell of the line and 1/2 elsewhere).  With face measures
// A_x = h_y h_z, A_y = h_x h_z, A_z = h_x h_y and V = h_x h_y h_z:
//   psi (sigma_t V + sum_a |O_a| A_a (1 + k_a)) = src + sum_a |O_a| A_a (T_a + k_a psi_a)
// where T_a is the upwind cell's outflow face value and psi_a its average (LMDG:
// k_a = 0, T_a = psi_a).  Per direction the sweep accumulates the weighted rows of the
// second block row of the reduced system: for a slope test function b_m,
//   xi_a      : O_a A_a (T_a - psi) + (eps sigma_a V / 3 + |O_a| A_a) c_a
//               + sum_{b != a} |O_b| A_b (c_a - c_a of the b-upwind cell) / 3
//   xi_a xi_b : (O_a A_a (c_b of the a-upwind cell - c_b) + O_b A_b (c_a of the
//               b-upwind cell - c_a)) / 3
//   xi eta zeta: 0
// (LMDG keeps only O_a A_a (psi_a - psi) on xi_a), plus w c_a for P_1 R (RLMDG).
// The standard scheme solves the 8 x 8 block of eq-Ljk for the trilinear moments c_m
// (m = b_x + 2 b_y + 4 b_z, basis prod_a xi_a^{b_a}), see cell_std3.
#include "internal.h"
#include "sweep_common.h"

namespace lmdg {
namespace {

template <int S> struct Traits3;
// NOUT: per-cell outputs; NF: values handed downwind per axis; NK: staged coefficients
// per cell; NA: per-source coefficient arrays of coef3_kernel.
//   STD   outputs w c_m (m = 0..7); traces: the four face moments of the outflow trace;
//         coefficients sigma_t V, a_0..a_7.
//   LMDG  outputs [P_0, xi, eta, zeta rows]; trace psi; coefficients sigma_t V, a, b_x,
//         b_y, b_z (src = a + |Ox| b_x + |Oy| b_y + |Oz| b_z).
//   RLMDG outputs [P_0, xi, eta, zeta, xi eta, xi zeta, eta zeta rows, P_1 R xi, eta,
//         zeta]; traces [outflow face value, two tangential slopes, cell value];
//         coefficients as LMDG plus eps sigma_a V / 3.
template <> struct Traits3<LMDG_SCHEME_STD> { static constexpr int NOUT = 8, NF = 4, NK = 9, NA = 8; };
template <> struct Traits3<LMDG_SCHEME_LMDG> { static constexpr int NOUT = 4, NF = 1, NK = 5, NA = 7; };
template <> struct Traits3<LMDG_SCHEME_RLMDG> { static constexpr int NOUT = 10, NF = 4, NK = 6, NA = 7; };

template <typename R>
struct Dir3 {
  R ao[3];   // |Omega_a|
  R aA[3];   // |Omega_a| A_a
  R oA[3];   // Omega_a A_a
  R woA[3];  // w Omega_a A_a   (FP32 RLMDG rows: the weight folded into the constants)
  R w3A[3];  // w |Omega_a| A_a / 3
  R w;
  int idx;
};

// 1 / d in the sweep: FP32 takes the hardware reciprocal (1 ulp), far inside the FP32
// sweep's accuracy; FP64 refines it (recip)
template <typename R>
__device__ __forceinline__ R recip3(R d) {
  if constexpr (sizeof(R) == 4)
    return __builtin_amdgcn_rcpf(d);
  else
    return recip(d);
}

__host__ __device__ constexpr int popc3(int m) { return (m & 1) + ((m >> 1) & 1) + ((m >> 2) & 1); }
// staged plane buffers of the sweep: planes p - L .. p + 1
__host__ __device__ constexpr int nbuf3(int L) { return L + 2; }
// (1/3)^(number of linear factors of mode m): the L2 norm squared of b_m on [-1,1]^3 / 8
template <typename R>
__device__ __forceinline__ constexpr R mass3(int m) {
  return popc3(m) == 0 ? R(1) : (popc3(m) == 1 ? R(1) / R(3) : (popc3(m) == 2 ? R(1) / R(9) : R(1) / R(27)));
}
// Index of a cell mode t without axis a among the four modes of a face normal to a:
// bit 0 the lower remaining axis, bit 1 the upper one.
__device__ __forceinline__ constexpr int face_idx(int a, int t) {
  return a == 0 ? (t >> 1) : (a == 1 ? ((t & 1) | ((t >> 1) & 2)) : (t & 3));
}
// The cell mode without axis a whose face index is f (inverse of face_idx).
__device__ __forceinline__ constexpr int face_mode(int a, int f) {
  return a == 0 ? (f << 1) : (a == 1 ? ((f & 1) | ((f & 2) << 1)) : f);
}

// Per-cell source coefficients shared by the eight octants, computed once per launch in
// FP64 and stored in the sweep precision R, so that the sweep stages six (nine) values
// per cell and octant instead of gathering the neighbourhood of every cell.
//
// LMDG/RLMDG, out [n_rhs][7][ncell]: a, then b_a for s_a = +1 and s_a = -1 per axis a
// (array 1 + 2 a + (s_a < 0)); then [2][ncell]: sigma_t V and eps sigma_a V / 3.
//   Plain form  M_0 x_0 + L_01 Sigma^T x_1 (+ Q~_0):
//     a = (sigma_s/eps) V x_0 + eps q V,  b_a = s_a A_a (slope_a(K) - slope_a(upwind)).
//   Defect form (L~_00 Sigma_0^T - M_0) x_0 - L_01 Sigma^T x_1 (the same operator with the
//   sigma_s/eps parts cancelled, as in the 2D kernel):
//     a = eps sigma_a V x_0 + eps q V,
//     b_a = -s_a A_a (slope_a(K) - slope_a(upwind)) + A_a (T_a(K) - T_a(upwind))
//   with T the outflow face value of x_0 along a (x_0 itself for LMDG; x_0 + k (x_0 -
//   x_0,up) for RLMDG; zero outside the mesh).  The upwind neighbour along a is the cell
//   at -s_a e_a; its distance from the inflow boundary decides k.
// STD, out [n_rhs][8][ncell]: a_m = (sigma_s/eps) V mass_m x_m (+ eps q V for m = 0),
// the plain form M Phi (+ Q) of eq-sndg-phi; then [1][ncell]: sigma_t V.
template <typename R, int S>
__global__ void coef3_kernel(Coef3Params P, R* __restrict__ out) {
  constexpr int NA = Traits3<S>::NA;
  const long long nc = P.ncell;
  const long long stride[3] = {1, P.n[0], (long long)P.n[0] * P.n[1]};
  // one cell per thread and loop trip, all sources in turn: the cell's indices are formed
  // once (32-bit divisions where the mesh allows; 64-bit ones cost several times more)
  for (long long cell = blockIdx.x * (long long)blockDim.x + threadIdx.x; cell < nc;
       cell += (long long)gridDim.x * blockDim.x) {
    int idx[3];
    if (nc <= 0xffffffffll) {
      const unsigned c = (unsigned)cell, n0 = (unsigned)P.n[0], n1 = (unsigned)P.n[1];
      const unsigned t = c / n0;
      idx[0] = (int)(c - t * n0);
      idx[1] = (int)(t % n1);
      idx[2] = (int)(t / n1);
    } else {
      idx[0] = (int)(cell % P.n[0]);
      idx[1] = (int)((cell / P.n[0]) % P.n[1]);
      idx[2] = (int)(cell / ((long long)P.n[0] * P.n[1]));
    }
    for (int rh = 0; rh < P.n_rhs; ++rh) {
      const double* x = P.x ? P.x + (long long)rh * 8 * nc : nullptr;
      const double qA = P.qA ? P.qA[(long long)rh * nc + cell] : 0.0;
      R* o = out + (long long)rh * NA * nc + cell;
      if constexpr (S == LMDG_SCHEME_STD) {
        const double scat = P.scatA[cell];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const double v = x ? scat * mass3<double>(m) * x[m * nc + cell] : 0.0;
          o[m * nc] = (R)(m == 0 ? v + qA : v);
        }
        if (rh == 0) out[(long long)P.n_rhs * NA * nc + cell] = (R)P.sigtA[cell];
      } else {
        const double x0 = x ? x[cell] : 0.0;
        o[0] = (R)((P.defect ? P.absA[cell] : P.scatA[cell]) * x0 + qA);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int sm = 1 << a;  // slope moment of axis a
#pragma unroll
          for (int sg = 0; sg < 2; ++sg) {
            const int sgn = sg ? -1 : 1;
            const int pos = sgn > 0 ? idx[a] : P.n[a] - 1 - idx[a];  // upwind cells inside the mesh
            double b = 0.0;
            if (x) {
              const long long up = cell - sgn * stride[a];
              const double u1 = pos >= 1 ? x[up] : 0.0;
              const double u2 = pos >= 2 ? x[up - sgn * stride[a]] : 0.0;
              const double sl = x[sm * nc + cell], slu = pos >= 1 ? x[sm * nc + up] : 0.0;
              const double ds = sgn * P.A[a] * (sl - slu);
              b = ds;
              if (P.defect) {
                double t = x0, tu = u1;
                if (S == LMDG_SCHEME_RLMDG) {
                  t = x0 + (pos == 0 ? 1.0 : 0.5) * (x0 - u1);
                  tu = pos > 0 ? u1 + (pos == 1 ? 1.0 : 0.5) * (u1 - u2) : 0.0;
                }
                b = -ds + P.A[a] * (t - tu);
              }
            }
            o[(1 + 2 * a + sg) * nc] = (R)b;
          }
        }
        if (rh == 0) {
          out[(long long)P.n_rhs * NA * nc + cell] = (R)P.sigtA[cell];
          out[((long long)P.n_rhs * NA + 1) * nc + cell] = (R)(P.absA[cell] * (1.0 / 3.0));
        }
      }
    }
  }
}

// Standard Q^1 cell (eq-Ljk in 3D): the 8 x 8 block sigma_t V M + streaming + outflow
// faces for the trilinear moments c, right-hand side a (8 source moments) plus the
// inflow traces.  With mass_m = (1/3)^{#linear factors of m} and for each axis a:
//   streaming  -int u Omega.grad b_n:  row n with bit a, column n - a: -2 O_a A_a mass_{n-a}
//   outflow    int_{xi_a = s_a} |O_a| u b_n:  rows and columns n, m that differ at most in
//              bit a: |O_a| A_a s_a^{b_a(n) + b_a(m)} mass_{n-a}
//   inflow     the upwind cell's outflow trace T (face moments over the other two axes)
//              enters row n as |O_a| A_a (-s_a)^{b_a(n)} mass_{n-a} T_{n-a}.
// The symmetric part of the block is positive definite, so elimination needs no pivoting.
// Outflow traces handed downwind along a: T_t = c_t + s_a c_{t+a} for the modes t without a.
template <typename R>
__device__ __forceinline__ void cell_std3(const Dir3<R>& d, R wa, const int si[3], const R* src, R sigV, const R* xin,
                                          const R* yin, const R* zin, R* xo, R* yo, R* zo, R* o, R* c) {
  R m[8][8], b[8];
#pragma unroll
  for (int n = 0; n < 8; ++n) {
#pragma unroll
    for (int k = 0; k < 8; ++k) m[n][k] = R(0);
    m[n][n] = sigV * mass3<R>(n);
    b[n] = src[n];
  }
  const R* tin[3] = {xin, yin, zin};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int bit = 1 << a;
    const R sg = R(si[a]);
#pragma unroll
    for (int n = 0; n < 8; ++n) {
      const int t = n & ~bit;
      const R fm = mass3<R>(t);
      if (n & bit) m[n][t] += R(-2) * d.oA[a] * fm;
      // outflow: columns t and t + a
      const R sn = (n & bit) ? sg : R(1);
      m[n][t] += d.aA[a] * sn * fm;
      m[n][t | bit] += d.aA[a] * sn * sg * fm;
      // inflow
      b[n] += d.aA[a] * ((n & bit) ? -sg : R(1)) * fm * tin[a][face_idx(a, t)];
    }
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const R inv = R(1) / m[k][k];
#pragma unroll
    for (int i = k + 1; i < 8; ++i) {
      const R f = m[i][k] * inv;
#pragma unroll
      for (int j = k + 1; j < 8; ++j) m[i][j] -= f * m[k][j];
      b[i] -= f * b[k];
    }
  }
#pragma unroll
  for (int k = 7; k >= 0; --k) {
    R acc = b[k];
#pragma unroll
    for (int j = k + 1; j < 8; ++j) acc -= m[k][j] * c[j];
    c[k] = acc / m[k][k];
  }
  R* tout[3] = {xo, yo, zo};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int bit = 1 << a;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const int t = face_mode(a, f);
      tout[a][f] = c[t] + R(si[a]) * c[t | bit];
    }
  }
#pragma unroll
  for (int n = 0; n < 8; ++n) o[n] = wa * c[n];
}

// Periods by which block b - 1 must lead block b: row r takes, in period p, the x trace
// of plane p - (r >> LCB), which block b - 1 produces in its period p - (r >> LCB) +
// ((CB - 1 + r) >> LCB) (the cell in its last column).
constexpr int x_lead3(int cb, int lcb) {
  int m = 0;
  for (int r = 0; r < kRows; ++r) {
    const int lead = ((cb - 1 + r) >> lcb) - (r >> lcb);
    m = lead > m ? lead : m;
  }
  return m;
}
static_assert(x_lead3(4, 2) == 1 && x_lead3(8, 3) == 1 && x_lead3(16, 4) == 1, "x traces of block b - 1");

// P1R: also the P_1 R rows of RLMDG (read by the recovery and by lmdg_sweep's output;
// operator applications and right-hand sides skip them).  PSI: angular fluxes stored.
template <typename R, int S, int MAXW, int CB, bool P1R, bool PSI>
__global__ void __launch_bounds__(64 * MAXW, 3) sweep3d_kernel(Sweep3Params<R> P) {
  constexpr int NOUT_ALL = Traits3<S>::NOUT;       // partial rows per cell (layout stride)
  constexpr int NOUT = (S == LMDG_SCHEME_RLMDG && !P1R) ? 7 : NOUT_ALL;  // rows produced
  constexpr int NOUTP = (NOUT + 3) & ~3;  // rows of red, padded to whole lane groups
  constexpr int NF = Traits3<S>::NF;
  constexpr int NK = Traits3<S>::NK;
  constexpr int NA = Traits3<S>::NA;
  constexpr int LCB = CB == 4 ? 2 : (CB == 8 ? 3 : 4);
  static_assert((1 << LCB) == CB, "CB is 4, 8 or 16");
  constexpr int CB16 = CB * kRows;
  constexpr int L = (kRows - 1 + CB - 1) / CB;  // periods by which row 15 trails row 0
  constexpr int NBUF = nbuf3(L);                // staged planes: p - L .. p and p + 1
  constexpr int XLEAD = x_lead3(CB, LCB);        // periods of block b - 1 ahead of block b
  constexpr int RING = NBUF * CB;               // staged cells per row (lambda modulo RING)
  constexpr int MAXC = (CB16 + 63) / 64;        // staged cells per thread (one wave at least)
  // y-trace values of a period per thread: CB ds NF of them over 64 ceil(ds / 4) threads
  constexpr int MAXE = (CB * NF + 15) / 16 > 0 ? (CB * NF + 15) / 16 : 1;
  constexpr bool RLM = S == LMDG_SCHEME_RLMDG;
  constexpr bool STDS = S == LMDG_SCHEME_STD;
  extern __shared__ unsigned char smem_raw[];
  __shared__ int s_item;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int W = blockDim.x >> 6;
  const int r = lane & 15;
  const int slot = wv * 4 + (lane >> 4);
  const long long nc = P.ncell;
  const int nx = P.nx, ny = P.ny, nz = P.nz, nstrips = P.nstrips, nblk = P.nblk;
  const long long nxy = (long long)nx * ny;
  const int ds = P.dslots;
  const double A[3] = {P.h[1] * P.h[2], P.h[0] * P.h[2], P.h[0] * P.h[1]};
  // LDS: red [CB][W][NOUTP][16] (+1 pad per step) | cbuf [RING][NK][16] | eds [CB][ds][NF]
  //      | ybuf [CB][ds][NF] (the top row's y traces of the period, written out after the steps)
  R* red = reinterpret_cast<R*>(smem_raw);
  // one step's block of red holds W x NOUTP x 16 values plus one pad, so that the
  // reduction's reads of consecutive steps fall in different banks
  const int red_tt = W * NOUTP * kRows + 1;
  R* cbuf = red + (size_t)CB * red_tt;
  R* eds = cbuf + (size_t)RING * NK * kRows;
  R* ybuf = eds + (size_t)CB * ds * NF;

  for (;;) {
    if (tid == 0) s_item = (int)(atomicAdd(P.ticket, 1u) - P.ticket_base);
    __syncthreads();
    const int item = s_item;
    if (item >= P.n_items) break;
    // item = ((s * nblk + b) * n_rhs + rhs) * 8 + octant: both items it waits for,
    // (s, b - 1) and (s - 1, b), come earlier
    const int o = item & 7;
    int rest = item >> 3;
    const int rh = rest % P.n_rhs;
    rest /= P.n_rhs;
    const int b = rest % nblk;
    const int s = rest / nblk;
    int si[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) si[a] = ((o >> a) & 1) ? -1 : 1;
    const long long ro = (long long)rh * 8 + o;
    R* const partr = P.part + ro * NOUT_ALL * nc;
    // [nz][nstrips][nblk][NF][ds][16]: a wave's lanes (16 rows x 4 slots) touch 256
    // consecutive bytes per trace value (agent-scope accesses go through to memory, so a
    // strided pattern would move whole lines for a quarter of their bytes)
    R* const xeb = P.xedge + ro * P.xedge_ostride;
    R* const yeb = P.yedge + ro * P.yedge_ostride;   // [nz + L][nstrips][nblk][CB][ds][NF]
    unsigned long long* const progr = P.prog + ro * (long long)nstrips * nblk;
    double* const psir = PSI ? P.psi + rh * P.psi_rstride : nullptr;
    const R* const cf_rh = P.coef + (long long)rh * NA * nc;
    const R* const cf_sh = P.coef + (long long)P.n_rhs * NA * nc;  // shared: sigma_t V (, eps sigma_a V / 3)

    Dir3<R> d;
    {
      const double* e = P.dirs + ((long long)o * ds + slot) * kDirStride;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        d.ao[a] = (R)fabs(e[a]);
        d.aA[a] = (R)(fabs(e[a]) * A[a]);
        d.oA[a] = (R)(e[a] * A[a]);
        d.woA[a] = (R)(e[3] * e[a] * A[a]);
        d.w3A[a] = (R)(e[3] * fabs(e[a]) * A[a] / 3.0);
      }
      d.w = (R)e[3];
      d.idx = (int)e[4];
    }
    const int jr = s * kRows + r;
    const bool row_ok = jr < ny;
    const int j = si[1] > 0 ? jr : ny - 1 - jr;
    const int c0 = b * CB;  // first column of the block (sweep order)
    const R ky = (jr == 0) ? R(1) : R(0.5);

    // coefficients of the cells of plane q of the block: loaded to registers (stage_load)
    // and stored to plane buffer q % NBUF (stage_store); cells outside the mesh get
    // sigma_t V = 1 and zero sources, so that every lane computes finite values
    R stg[MAXC][NK];
    auto stage_load = [&](int q) {
#pragma unroll
      for (int mc = 0; mc < MAXC; ++mc) {
        const int e = tid + mc * (int)blockDim.x;
        const int cl = e & (CB - 1), rr = e >> LCB;
        const int c = c0 + cl, jr2 = s * kRows + rr;
        const bool in = e < CB16 && c < nx && jr2 < ny && q < nz;
#pragma unroll
        for (int k = 0; k < NK; ++k) stg[mc][k] = (k == 0) ? R(1) : R(0);
        if (in) {
          const int i2 = si[0] > 0 ? c : nx - 1 - c;
          const int j2 = si[1] > 0 ? jr2 : ny - 1 - jr2;
          const int k2 = si[2] > 0 ? q : nz - 1 - q;
          const long long cell = (long long)k2 * nxy + (long long)j2 * nx + i2;
          stg[mc][0] = cf_sh[cell];
          if constexpr (STDS) {
#pragma unroll
            for (int m = 0; m < 8; ++m) stg[mc][1 + m] = cf_rh[m * nc + cell];
          } else {
            stg[mc][1] = cf_rh[cell];
#pragma unroll
            for (int a = 0; a < 3; ++a) stg[mc][2 + a] = cf_rh[(1 + 2 * a + (si[a] < 0)) * nc + cell];
            if constexpr (RLM) stg[mc][5] = cf_sh[nc + cell];
          }
        }
      }
    };
    auto stage_store = [&](int buf) {
#pragma unroll
      for (int mc = 0; mc < MAXC; ++mc) {
        const int e = tid + mc * (int)blockDim.x;
        if (e < CB16) {
          const int cl = e & (CB - 1), rr = e >> LCB;
          R* dst = cbuf + (size_t)(buf * CB + cl) * NK * kRows + rr;
#pragma unroll
          for (int k = 0; k < NK; ++k) dst[k * kRows] = stg[mc][k];
        }
      }
    };

    R zreg[CB][NF], xin[NF], yprev[NF], xe[NF], xsave[NF];
    // FP32: x traces block b - 1 stored in period p + 1, loaded in period p by every row
    // (one whole 64-byte run per slot); rows that take them in period p + 1 hold them
    R xhold[NF];
    unsigned long long seen_b = 0, seen_s = 0;  // progress words last read (thread 0)
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      xin[f] = yprev[f] = xsave[f] = xhold[f] = R(0);
#pragma unroll
      for (int u = 0; u < CB; ++u) zreg[u][f] = R(0);
    }
    // plane buffers other than the first hold neutral values until staged (rows that
    // trail into planes before the first read them)
    for (int e = CB * NK * kRows + tid; e < RING * NK * kRows; e += blockDim.x)
      cbuf[e] = ((e / kRows) % NK == 0) ? R(1) : R(0);
    stage_load(0);
    stage_store(0);
    int pb = 0;  // p % NBUF
    for (int p = 0; p < nz + L; ++p) {
      // wait until (s, b - 1) has completed period p + XLEAD and (s - 1, b) period p + L
      // (both clamped to the last period): thread 0 keeps the progress words it last read
      // and reads a word again only while that falls short, both words at once
      if (tid == 0 && (s > 0 || b > 0)) {
        const unsigned long long tag = (P.epoch + P.wait_bias) << 32;
        const unsigned long long tb = tag | (unsigned long long)min(p + 1 + XLEAD, nz + L);
        const unsigned long long ts = tag | (unsigned long long)min(p + 1 + L, nz + L);
        const unsigned long long* fb = progr + (long long)s * nblk + (b - 1);
        const unsigned long long* fs = progr + (long long)(s - 1) * nblk + b;
        long long spins = 0;
        while ((b > 0 && seen_b < tb) || (s > 0 && seen_s < ts)) {
          if (b > 0 && seen_b < tb) seen_b = load_agent(fb);
          if (s > 0 && seen_s < ts) seen_s = load_agent(fs);
          if ((b > 0 && seen_b < tb) || (s > 0 && seen_s < ts)) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > P.spin_limit) { atomicOr(P.err, 1); break; }
          }
        }
      }
      __syncthreads();
      // y traces of strip s - 1 at plane p for the block's columns (row 0's inflow) and x
      // traces of block b - 1 for this row at the plane where the row enters the block,
      // issued together: every address is clamped into the buffers and values that do not
      // exist (first strip or block, planes outside the mesh, ragged columns) are replaced
      // by zero afterwards, so that the loads carry no branches and one memory latency
      // covers both before the y traces go to LDS
      {
        const int ne = CB * ds * NF;
        const int ne_in = (s > 0 && p < nz) ? min(CB, nx - c0) * ds * NF : 0;  // columns inside the mesh
        // row 15 of strip s - 1 passed the cell in column 0 at the last step of its period
        // p + L - 1 and the cells in columns 1 .. CB - 1 at steps 0 .. CB - 2 of period p + L
        const long long yblk = (long long)max(s - 1, 0) * nblk + b;
        const R* ya = yeb + ((long long)min(p + L - 1, nz + L - 1) * nstrips * nblk + yblk) * ne + (CB - 1) * ds * NF;
        const R* yb = yeb + ((long long)min(p + L, nz + L - 1) * nstrips * nblk + yblk) * ne - ds * NF;
        R ev[MAXE];
#pragma unroll
        for (int k = 0; k < MAXE; ++k) {
          const int e = tid + k * (int)blockDim.x;
          const R v = load_agent(e < ne_in ? (e < ds * NF ? ya : yb) + e : yeb);
          ev[k] = e < ne_in ? v : R(0);
        }
        // row r takes the trace of plane p - (r >> LCB), which block b - 1 stored in its
        // period p + XL(r)
        const int qx = p - (r >> LCB);
        const bool ok = b > 0 && row_ok && qx >= 0 && qx < nz;
        if constexpr (sizeof(R) == 4) {
          const bool later = ((r + CB - 1) >> LCB) == (r >> LCB);
          const long long xrow = ((long long)s * nblk + max(b - 1, 0)) * kRows * ds * NF + slot * kRows + r;
          const R* xsrc = xeb + (long long)min(p + 1, nz + L - 1) * nstrips * nblk * kRows * ds * NF + xrow;
          R xl[NF];
#pragma unroll
          for (int f = 0; f < NF; ++f) xl[f] = load_agent(xsrc + f * ds * kRows);
          if (p == 0) {  // the rows that take period 0's traces in period 0
#pragma unroll
            for (int f = 0; f < NF; ++f) xhold[f] = load_agent(xeb + xrow + f * ds * kRows);
          }
#pragma unroll
          for (int f = 0; f < NF; ++f) {
            xe[f] = ok ? (later ? xhold[f] : xl[f]) : R(0);
            xhold[f] = xl[f];
          }
        } else {
          const int px = min(p + ((r + CB - 1) >> LCB) - (r >> LCB), nz + L - 1);
          const R* xsrc = xeb + (((long long)px * nstrips + s) * nblk + max(b - 1, 0)) * kRows * ds * NF + slot * kRows + r;
#pragma unroll
          for (int f = 0; f < NF; ++f) {
            const R v = load_agent(xsrc + f * ds * kRows);
            xe[f] = ok ? v : R(0);
          }
        }
#pragma unroll
        for (int k = 0; k < MAXE; ++k) {
          const int e = tid + k * (int)blockDim.x;
          if (e < ne) eds[e] = ev[k];
        }
      }
      lds_barrier();  // staged y traces visible

      // the row index passes through an empty asm once per period, so that the per-step
      // values derived from it are recomputed here instead of being held in registers
      // across the whole item
      int rp = r;
      asm volatile("" : "+v"(rp));
      const int lbase = p * CB - rp;    // the lane's sequence index at step 0
      const int rc = rp & (CB - 1);     // step at which its cell is in the block's first column
      const int slot0 = (lbase + RING) % RING;  // its staged slot at step 0 (lbase > -RING)
      // Cells outside the mesh (planes before 0 or from nz on, ragged rows and columns)
      // are computed like the others from the neutral staged values; their rows and
      // traces are never read.  Before plane 0 every source and inflow is zero, so those
      // cells hand zero traces on, and plane 0 finds its zero z-inflow in the registers.
#pragma unroll
      for (int u = 0; u < CB; ++u) {
          const int lam = lbase + u;                    // sequence index: plane * CB + column
          const bool first = rc == u;                   // column 0 of the block
          const bool last = rc == ((u + 1) & (CB - 1)); // column CB - 1 of the block
          const bool plane0 = (unsigned)lam < (unsigned)CB;
          int sl;
          if constexpr ((RING & (RING - 1)) == 0) {
            sl = lam & (RING - 1);
          } else {
            sl = slot0 + u;
            if (sl >= RING) sl -= RING;
          }
          const R* cf = cbuf + (size_t)sl * (NK * kRows) + r;
          // y-inflow: the row below (DPP row shift); row 0 takes the y-outflow of strip
          // s - 1.  FP32: every lane reads the staged trace and the shift keeps it in row 0;
          // FP64: row 0 alone reads it (four doubles per lane and step cost more LDS
          // bandwidth than the select saves)
          R xi[NF], yd[NF], zi[NF];
#pragma unroll
          for (int f = 0; f < NF; ++f) {
            xi[f] = first ? xe[f] : xin[f];
            if constexpr (sizeof(R) == 4) {
              yd[f] = shr1_or(yprev[f], eds[(u * ds + slot) * NF + f]);
            } else {
              const R v = shr1(yprev[f]);
              yd[f] = (r == 0) ? eds[(u * ds + slot) * NF + f] : v;
            }
            zi[f] = zreg[u][f];
          }
          R o[NOUT_ALL], xo[NF], yo[NF], zo[NF];
          // angular fluxes are stored only for cells inside the mesh
          auto in_mesh = [&](int& q_out, int& c_out) {
            q_out = lam >> LCB;
            c_out = c0 + (lam & (CB - 1));
            return row_ok && q_out >= 0 && q_out < nz && c_out < nx;
          };
          if constexpr (STDS) {
            R src[8], cm[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) src[m] = cf[(1 + m) * kRows];
            cell_std3<R>(d, d.w, si, src, cf[0], xi, yd, zi, xo, yo, zo, o, cm);
            if constexpr (PSI) {
              int q, c;
              if (in_mesh(q, c) && d.idx >= 0) {
                const int i = si[0] > 0 ? c : nx - 1 - c;
                const int kk = si[2] > 0 ? q : nz - 1 - q;
                const long long cell = (long long)kk * nxy + (long long)j * nx + i;
#pragma unroll
                for (int m = 0; m < 8; ++m) psir[((long long)d.idx * 8 + m) * nc + cell] = (double)cm[m];
              }
            }
          } else {
            const R sig = cf[0];
            const R src = cf[kRows] + d.ao[0] * cf[2 * kRows] + d.ao[1] * cf[3 * kRows] + d.ao[2] * cf[4 * kRows];
            const R w = d.w;
            R psi;
            if constexpr (!RLM) {
              const R inv = recip3(sig + d.aA[0] + d.aA[1] + d.aA[2]);
              psi = (src + d.aA[0] * xi[0] + d.aA[1] * yd[0] + d.aA[2] * zi[0]) * inv;
              xo[0] = yo[0] = zo[0] = psi;
              o[0] = w * psi;
              o[1] = w * d.oA[0] * (xi[0] - psi);
              o[2] = w * d.oA[1] * (yd[0] - psi);
              o[3] = w * d.oA[2] * (zi[0] - psi);
            } else {
              // traces per axis: [outflow face value, two tangential slopes, cell value];
              // tangential slopes in axis order: x carries (c_y, c_z), y (c_x, c_z), z (c_x, c_y)
              const R kx = (b == 0 && first) ? R(1) : R(0.5);
              const R kz = plane0 ? R(1) : R(0.5);
              const R third = R(1) / R(3);
              const R inv = recip3(sig + d.aA[0] * (R(1) + kx) + d.aA[1] * (R(1) + ky) + d.aA[2] * (R(1) + kz));
              psi = (src + d.aA[0] * (xi[0] + kx * xi[3]) + d.aA[1] * (yd[0] + ky * yd[3]) +
                     d.aA[2] * (zi[0] + kz * zi[3])) *
                    inv;
              const R cx = R(si[0]) * kx * (psi - xi[3]);
              const R cy = R(si[1]) * ky * (psi - yd[3]);
              const R cz = R(si[2]) * kz * (psi - zi[3]);
              xo[0] = psi + kx * (psi - xi[3]);
              xo[1] = cy;
              xo[2] = cz;
              xo[3] = psi;
              yo[0] = psi + ky * (psi - yd[3]);
              yo[1] = cx;
              yo[2] = cz;
              yo[3] = psi;
              zo[0] = psi + kz * (psi - zi[3]);
              zo[1] = cx;
              zo[2] = cy;
              zo[3] = psi;
              // eps sigma_a V / 3: sigma_t V / 3 of L_11 R minus (sigma_s/eps) V / 3 of M_1 P_1 R
              const R sV3 = cf[5 * kRows];
              o[0] = w * psi;
              if constexpr (sizeof(R) == 4) {
                // FP32: the weight enters through the direction constants woA, w3A (fewer
                // instructions; FP64 keeps the product form, which needs fewer registers)
                const R wsV3 = w * sV3;
                o[1] = d.woA[0] * (xi[0] - psi) + (wsV3 + R(3) * d.w3A[0]) * cx + d.w3A[1] * (cx - yd[1]) +
                       d.w3A[2] * (cx - zi[1]);
                o[2] = d.woA[1] * (yd[0] - psi) + (wsV3 + R(3) * d.w3A[1]) * cy + d.w3A[0] * (cy - xi[1]) +
                       d.w3A[2] * (cy - zi[2]);
                o[3] = d.woA[2] * (zi[0] - psi) + (wsV3 + R(3) * d.w3A[2]) * cz + d.w3A[0] * (cz - xi[2]) +
                       d.w3A[1] * (cz - yd[2]);
                o[4] = third * (d.woA[0] * (xi[1] - cy) + d.woA[1] * (yd[1] - cx));
                o[5] = third * (d.woA[0] * (xi[2] - cz) + d.woA[2] * (zi[1] - cx));
                o[6] = third * (d.woA[1] * (yd[2] - cz) + d.woA[2] * (zi[2] - cy));
              } else {
                o[1] = w * (d.oA[0] * (xi[0] - psi) + (sV3 + d.aA[0]) * cx +
                            third * (d.aA[1] * (cx - yd[1]) + d.aA[2] * (cx - zi[1])));
                o[2] = w * (d.oA[1] * (yd[0] - psi) + (sV3 + d.aA[1]) * cy +
                            third * (d.aA[0] * (cy - xi[1]) + d.aA[2] * (cy - zi[2])));
                o[3] = w * (d.oA[2] * (zi[0] - psi) + (sV3 + d.aA[2]) * cz +
                            third * (d.aA[0] * (cz - xi[2]) + d.aA[1] * (cz - yd[2])));
                o[4] = w * third * (d.oA[0] * (xi[1] - cy) + d.oA[1] * (yd[1] - cx));
                o[5] = w * third * (d.oA[0] * (xi[2] - cz) + d.oA[2] * (zi[1] - cx));
                o[6] = w * third * (d.oA[1] * (yd[2] - cz) + d.oA[2] * (zi[2] - cy));
              }
              if constexpr (P1R) {
                o[7] = w * cx;
                o[8] = w * cy;
                o[9] = w * cz;
              }
            }
            if constexpr (PSI) {
              int q, c;
              if (in_mesh(q, c) && d.idx >= 0) {
                const int i = si[0] > 0 ? c : nx - 1 - c;
                const int kk = si[2] > 0 ? q : nz - 1 - q;
                psir[(long long)d.idx * nc + (long long)kk * nxy + (long long)j * nx + i] = (double)psi;
              }
            }
          }
#pragma unroll
          for (int f = 0; f < NF; ++f) {
            xin[f] = xo[f];
            yprev[f] = yo[f];
            zreg[u][f] = zo[f];
            xsave[f] = last ? xo[f] : xsave[f];
            // taken here: otherwise the selects sink below the last step and every
            // step's outflow stays live across the period
            asm volatile("" : "+v"(xsave[f]));
          }
          // top row: y traces for strip s + 1, staged in LDS for one store pass per period
          if (r == kRows - 1) {
#pragma unroll
            for (int f = 0; f < NF; ++f) ybuf[(u * ds + slot) * NF + f] = yo[f];
          }
          // sums over the four direction slots of the wave, four rows at a time: lane
          // group g receives row m0 + g
          R om[NOUTP];
#pragma unroll
          for (int m = 0; m < NOUTP; ++m) om[m] = m < NOUT ? o[m < NOUT ? m : 0] : R(0);
#pragma unroll
          for (int m0 = 0; m0 < NOUTP; m0 += 4) {
            const R v = quad_sum4(om[m0], om[m0 + 1], om[m0 + 2], om[m0 + 3]);
            red[u * red_tt + (wv * NOUTP + m0 + (lane >> 4)) * kRows + r] = v;
          }
          // keep each step's loads next to its arithmetic (bounds the registers held)
          __builtin_amdgcn_sched_barrier(0);
          // the next plane's coefficients: issued after the first step, whose x-inflow
          // needs the x traces above, and in flight through the other steps
          if (u == 0 && p + 1 < nz) stage_load(p + 1);
      }
      // y traces of the period's top-row cells for strip s + 1 (row 15 handled the cell
      // lambda = u - 15 at step u), stored under the period in one contiguous run (cells
      // outside the mesh hold finite values nobody reads)
      lds_barrier();
      if (s + 1 < nstrips) {
        const int ne = CB * ds * NF;
        R* dst = yeb + (((long long)p * nstrips + s) * nblk + b) * ne;
        for (int e = tid; e < ne; e += blockDim.x) store_agent(dst + e, ybuf[e]);
      }
      // x traces for block b + 1: the period's cell in the block's last column, stored
      // under the period for every row (rows whose cell lies outside the mesh hold finite
      // values nobody reads), so that each wave writes whole 64-byte runs of 16 rows
      if (b + 1 < nblk) {
        R* dst = xeb + (((long long)p * nstrips + s) * nblk + b) * kRows * ds * NF + slot * kRows + r;
#pragma unroll
        for (int f = 0; f < NF; ++f) store_agent(dst + f * ds * kRows, xsave[f]);
      }
      // the next plane's coefficients to LDS before the progress word: the write-through of
      // the trace stores above completes meanwhile
      const int pb1 = (pb + 1 == NBUF) ? 0 : pb + 1;
      if (p + 1 < nz) stage_store(pb1);
      // publish: periods 0 .. p are finished by every row of the block (their trace stores
      // included); waves wait for their own stores before the barrier
      const bool publish = s + 1 < nstrips || b + 1 < nblk;
      if (publish) __builtin_amdgcn_s_waitcnt(kWaitVmem);
      __syncthreads();
      if (tid == 0 && publish) store_agent(progr + (long long)s * nblk + b, (P.epoch << 32) | (unsigned long long)(p + 1));
      // the period's outputs after the progress word (the wait before it covers the trace
      // stores only): one cell per (row, column of the block) and thread, its NOUT rows
      // summed over the waves; the next period writes red after its first barrier
      for (int t = tid; t < CB16; t += blockDim.x) {
        const int cl = t & (CB - 1), rr = t >> LCB;
        const int u = (rr + cl) & (CB - 1);
        const int q = p + ((u - rr) >> LCB);
        const int c = c0 + cl;
        const int jr2 = s * kRows + rr;
        if (q >= 0 && q < nz && c < nx && jr2 < ny) {
          const R* src = red + u * red_tt + rr;
          const int i = si[0] > 0 ? c : nx - 1 - c;
          const int jj = si[1] > 0 ? jr2 : ny - 1 - jr2;
          const int kk = si[2] > 0 ? q : nz - 1 - q;
          R acc[NOUT];
#pragma unroll
          for (int m = 0; m < NOUT; ++m) acc[m] = src[m * kRows];
          for (int w2 = 1; w2 < W; ++w2) {
#pragma unroll
            for (int m = 0; m < NOUT; ++m) acc[m] += src[(w2 * NOUTP + m) * kRows];
          }
          R* dst = partr + (long long)kk * nxy + (long long)jj * nx + i;
#pragma unroll
          for (int m = 0; m < NOUT; ++m) dst[(long long)m * nc] = acc[m];
        }
      }
      pb = pb1;
    }
    __syncthreads();
  }
}

template <typename R, int S, bool P1R>
size_t lds_bytes3(int cb, int W, int dslots) {
  constexpr int NOUT = (S == LMDG_SCHEME_RLMDG && !P1R) ? 7 : Traits3<S>::NOUT;
  constexpr int NOUTP = (NOUT + 3) & ~3;
  const int L = (kRows - 1 + cb - 1) / cb;
  return ((size_t)cb * (W * NOUTP * kRows + 1) + (size_t)nbuf3(L) * Traits3<S>::NK * cb * kRows +
          (size_t)2 * cb * dslots * Traits3<S>::NF) *
         sizeof(R);
}

// Work items the GPU holds at once for one instantiation (occupancy query, cached).
template <typename R, int S, int MAXW, int CB, bool P1R, bool PSI>
int resident_blocks(int threads, size_t lds) {
  static int per_cu = -1;
  static size_t per_cu_lds = 0;
  if (per_cu < 0 || per_cu_lds != lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep3d_kernel<R, S, MAXW, CB, P1R, PSI>, threads, lds) !=
            hipSuccess ||
        nb < 1)
      nb = 1;
    per_cu = nb;
    per_cu_lds = lds;
  }
  return per_cu;
}

template <typename R, int S, int MAXW, int CB, bool P1R, bool PSI>
int launch_kernel3(lmdg_handle* h, const Sweep3Params<R>& P, int W, hipStream_t st) {
  const size_t lds = lds_bytes3<R, S, P1R>(CB, W, h->dslots);
  if (lds > 160 * 1024)
    return set_error(h, LMDG_UNSUPPORTED, "direction set too large for the 3D sweep's LDS staging");
  const int per_cu = resident_blocks<R, S, MAXW, CB, P1R, PSI>(64 * W, lds);
  const int grid = (int)std::min<long long>(P.n_items, (long long)per_cu * h->n_cu);
  hipLaunchKernelGGL((sweep3d_kernel<R, S, MAXW, CB, P1R, PSI>), dim3(grid), dim3(64 * W), lds, st, P);
  h->ticket_base += (unsigned)(P.n_items + grid);
  return LMDG_OK;
}

// Edge traces are stored per period of the producing item: nz + L periods, L = ceil(15 / CB).
constexpr int x_periods_extra3(int cb) { return (kRows - 1 + cb - 1) / cb; }

// Column block width: 8 for FP32 sweeps, 4 for FP64 (the register ring holds CB x NF
// values; wider blocks raise the register count past three waves per SIMD).
constexpr int kMinBlockCols3 = 4;
template <typename R>
constexpr int block_cols3() { return sizeof(R) == 4 ? 8 : 4; }
static_assert(block_cols3<float>() >= kMinBlockCols3 && block_cols3<double>() >= kMinBlockCols3, "workspace sizing");

template <typename R, int S, int MAXW, int CB>
int launch_kernel3_sel(lmdg_handle* h, const Sweep3Params<R>& P, int W, bool p1r, hipStream_t st) {
  if (P.psi) return launch_kernel3<R, S, MAXW, CB, true, true>(h, P, W, st);
  if (p1r || S != LMDG_SCHEME_RLMDG) return launch_kernel3<R, S, MAXW, CB, true, false>(h, P, W, st);
  return launch_kernel3<R, S, MAXW, CB, false, false>(h, P, W, st);
}

template <typename R, int S>
int launch3_typed(lmdg_handle* h, const double* x, bool use_q, double* psi, hipStream_t st, bool defect, bool p1r) {
  constexpr int CB = block_cols3<R>();
  constexpr int NF = Traits3<S>::NF;
  constexpr int NA = Traits3<S>::NA;
  const int W = h->waves;
  Sweep3Params<R> P;
  P.nx = (int)h->n[0];
  P.ny = (int)h->n[1];
  P.nz = (int)h->n[2];
  P.nstrips = h->nstrips;
  P.nblk = (P.nx + CB - 1) / CB;
  P.dslots = h->dslots;
  P.n_rhs = h->n_rhs;
  P.n_items = 8 * P.nstrips * P.nblk * h->n_rhs;
  for (int a = 0; a < 3; ++a) P.h[a] = h->h[a];
  P.ncell = h->ncell;
  P.dirs = h->d_dirs;
  // coefficients of every source in the sweep precision
  R* coef = reinterpret_cast<R*>(h->ws.zbuf);
  {
    Coef3Params C;
    for (int a = 0; a < 3; ++a) C.n[a] = (int)h->n[a];
    C.n_rhs = h->n_rhs;
    C.defect = defect ? 1 : 0;
    C.ncell = h->ncell;
    C.A[0] = h->h[1] * h->h[2];
    C.A[1] = h->h[0] * h->h[2];
    C.A[2] = h->h[0] * h->h[1];
    C.x = x;
    C.qA = use_q ? (h->src0 ? h->src0 : h->d_qA) : nullptr;
    C.sigtA = h->d_sigtA;
    C.scatA = h->d_scatA;
    C.absA = h->d_absA;
    const long long n = h->ncell;  // one thread per cell, all sources
    const int g = (int)std::min<long long>(std::max<long long>((n + 255) / 256, 1), 8192);
    hipLaunchKernelGGL((coef3_kernel<R, S>), dim3(g), dim3(256), 0, st, C, coef);
    (void)NA;
  }
  P.coef = coef;
  P.part = reinterpret_cast<R*>(h->ws.part);
  h->last_nsl = 8;
  P.xedge = reinterpret_cast<R*>(h->ws.edge);
  P.xedge_ostride = (long long)(P.nz + x_periods_extra3(CB)) * P.nstrips * P.nblk * kRows * h->dslots * NF;
  P.yedge = P.xedge + 8LL * h->n_rhs * P.xedge_ostride;
  P.yedge_ostride = (long long)(P.nz + x_periods_extra3(CB)) * P.nstrips * P.nblk * CB * h->dslots * NF;
  P.psi = psi;
  P.psi_rstride = (long long)h->ndir * (S == LMDG_SCHEME_STD ? 8 : 1) * h->ncell;
  P.prog = h->ws.prog;
  P.ticket = h->ws.ticket;
  P.err = h->ws.err;
  P.epoch = h->epoch;
  P.ticket_base = h->ticket_base;
  P.spin_limit = h->spin_limit;
  P.wait_bias = h->wait_bias;
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
  const int rc = W <= 4 ? launch_kernel3_sel<R, S, 4, CB>(h, P, W, p1r, st)
                        : launch_kernel3_sel<R, S, kMaxWaves, CB>(h, P, W, p1r, st);
  if (rc != LMDG_OK) return rc;
  if (ev_end) hipEventRecord(ev_end, st);
  h->epoch += 1;
  return check_hip(h, hipGetLastError(), "sweep launch");
}

}  // namespace

// Workspace of the 3D sweeps per right-hand side (the handle sizes it for the narrowest
// column blocks, FP64 values and four trace values): edge traces (x then y), per-cell
// coefficients, progress words.
size_t sweep3d_edge_bytes(const lmdg_handle* h) {
  const long long nblk = (h->n[0] + kMinBlockCols3 - 1) / kMinBlockCols3;
  const long long nz = h->n[2];
  return (size_t)8 * h->nstrips * (nz + x_periods_extra3(kMinBlockCols3)) * nblk * (kRows + kMinBlockCols3) *
         h->dslots * 4 * sizeof(double);
}
size_t sweep3d_coef_bytes(const lmdg_handle* h) { return (size_t)9 * h->ncell * sizeof(double); }
size_t sweep3d_prog_words(const lmdg_handle* h) {
  return (size_t)8 * h->nstrips * ((h->n[0] + kMinBlockCols3 - 1) / kMinBlockCols3);
}

int launch_sweep3d(lmdg_handle* h, int scheme, int prec, const double* x, bool use_q, double* psi, hipStream_t st,
                   bool defect, bool p1r) {
  if (scheme == LMDG_SCHEME_STD) {
    // the standard scheme takes the plain form M Phi (+ Q) of eq-sndg-phi
    return prec == LMDG_PREC_FP64 ? launch3_typed<double, LMDG_SCHEME_STD>(h, x, use_q, psi, st, false, true)
                                  : launch3_typed<float, LMDG_SCHEME_STD>(h, x, use_q, psi, st, false, true);
  }
  if (prec == LMDG_PREC_FP64)
    return scheme == LMDG_SCHEME_LMDG ? launch3_typed<double, LMDG_SCHEME_LMDG>(h, x, use_q, psi, st, defect, p1r)
                                      : launch3_typed<double, LMDG_SCHEME_RLMDG>(h, x, use_q, psi, st, defect, p1r);
  return scheme == LMDG_SCHEME_LMDG ? launch3_typed<float, LMDG_SCHEME_LMDG>(h, x, use_q, psi, st, defect, p1r)
                                    : launch3_typed<float, LMDG_SCHEME_RLMDG>(h, x, use_q, psi, st, defect, p1r);
}

}  // namespace lmdg
