// Transport sweeps of the low-memory schemes on a uniform 3D Cartesian mesh (gfx950).
//
// The 2D decomposition (sweep2d.hip) extended by one axis: a work item is
// (octant o, plane kz in sweep order, strip s of 16 y-rows, right-hand side); the
// workgroup holds every direction slot of the octant, lanes = 16 rows x 4 slots, and
// the x axis is walked in skewed steps (row r handles column t - r at step t).
// Upwind values arrive from three sides:
//   x  the lane's own previous cell (registers);
//   y  the lane below through one DPP row shift, row 0 from the strip-edge buffer
//      written by strip s - 1 of the same plane;
//   z  the plane below: every cell writes its z-outflow traces to a two-plane ring
//      buffer; plane kz stages the traces of plane kz - 1 for a chunk in LDS.
// An item waits for (kz, s - 1) and (kz - 1, s) to have finished the columns of the
// chunk (epoch-tagged progress words, bounded spin).  The ring buffer is safe with two
// planes: plane kz overwrites the slot that plane kz - 1 reads only at columns that
// plane kz - 1 has already published, i.e. finished reading.
//
// Local solves follow Sec. 3.2 (L_00, scalar per cell and direction) and Sec. 3.3
// (L~_00 = L_00 + L_01 R with the upwind slopes c_a = s_a k_a (psi - psi_up,a),
// k_a = 1 in the inflow cell of the line and 1/2 elsewhere).  With face measures
// A_x = h_y h_z, A_y = h_x h_z, A_z = h_x h_y and V = h_x h_y h_z:
//   psi (sigma_t V + sum_a |O_a| A_a (1 + k_a)) = src + sum_a |O_a| A_a (T_a + k_a psi_a)
// where T_a is the upwind cell's outflow face value and psi_a its average (LMDG:
// k_a = 0, T_a = psi_a).  Per direction the sweep accumulates the weighted rows of
// the second block row of the reduced system: for a slope test function b_m,
//   xi_a      : O_a A_a (T_a - psi) + (sigma_t V / 3 + |O_a| A_a) c_a
//               + sum_{b != a} |O_b| A_b (c_a - c_a of the b-upwind cell) / 3
//   xi_a xi_b : (O_a A_a (c_b of the a-upwind cell - c_b) + O_b A_b (c_a of the
//               b-upwind cell - c_a)) / 3
//   xi eta zeta: 0
// (LMDG keeps only O_a A_a (psi_a - psi) on xi_a), plus w c_a for P_1 R (RLMDG).
#include "internal.h"
#include "sweep_common.h"

namespace lmdg {
namespace {

template <int S> struct Traits3;
// NOUT: per-cell outputs [P_0, xi, eta, zeta rows (, xi eta, xi zeta, eta zeta rows,
// P_1 R xi, eta, zeta)]; NF: values handed downwind per axis; NRAW: FP64 inputs per cell
// NC: staged values per cell: sigma_t V, the source coefficients a, b_x, b_y, b_z, and for
// RLMDG eps sigma_a V / 3 (the slope mass term of the second block row)
template <> struct Traits3<LMDG_SCHEME_LMDG> { static constexpr int NOUT = 4, NF = 1, NC = 5; };
template <> struct Traits3<LMDG_SCHEME_RLMDG> { static constexpr int NOUT = 10, NF = 4, NC = 6; };
constexpr int kNRAW3 = 17;
constexpr int kMAXC3 = 2;   // staged cells per thread
constexpr int kStepGroup3 = 2;  // steps per unrolled group (measured best on gfx950)

template <typename R>
struct Dir3 {
  R ao[3];   // |Omega_a|
  R aA[3];   // |Omega_a| A_a
  R oA[3];   // Omega_a A_a
  R w;
  int idx;
};

// Raw FP64 inputs of one cell: x_0 at the cell and at its upwind and second-upwind
// neighbours along x, y, z; the slope moments xi, eta, zeta of x_1 at the cell and
// the upwind neighbour along the same axis; the four material values.  Zero outside.
template <typename R>
__device__ __forceinline__ void raw_load3_impl(const Sweep3Params<R>& P, const double* x, const double* qA,
                                               const int si[3], int c, int jr, int kz, double* raw) {
#pragma unroll
  for (int k = 0; k < kNRAW3; ++k) raw[k] = 0.0;
  if (c < 0 || c >= P.nx || jr >= P.ny) return;
  const long long nx = P.nx, nxy = (long long)P.nx * P.ny, nc = P.ncell;
  const int i = si[0] > 0 ? c : P.nx - 1 - c;
  const int j = si[1] > 0 ? jr : P.ny - 1 - jr;
  const int k = si[2] > 0 ? kz : P.nz - 1 - kz;
  const long long cell = (long long)k * nxy + (long long)j * nx + i;
  const long long dx = si[0], dy = si[1] * nx, dz = si[2] * nxy;  // cell - d: upwind
  if (x) {
    raw[0] = x[cell];
    if (c > 0) raw[1] = x[cell - dx];
    if (c > 1) raw[2] = x[cell - 2 * dx];
    if (jr > 0) raw[3] = x[cell - dy];
    if (jr > 1) raw[4] = x[cell - 2 * dy];
    if (kz > 0) raw[5] = x[cell - dz];
    if (kz > 1) raw[6] = x[cell - 2 * dz];
    raw[7] = x[1 * nc + cell];
    if (c > 0) raw[8] = x[1 * nc + cell - dx];
    raw[9] = x[2 * nc + cell];
    if (jr > 0) raw[10] = x[2 * nc + cell - dy];
    raw[11] = x[4 * nc + cell];
    if (kz > 0) raw[12] = x[4 * nc + cell - dz];
  }
  raw[13] = P.sigtA[cell];
  raw[14] = P.absA[cell];
  raw[15] = P.scatA[cell];
  raw[16] = qA ? qA[cell] : 0.0;
}

// Source coefficients of one cell (FP64), src = a + |Ox| b_x + |Oy| b_y + |Oz| b_z.
// Plain form M_0 x_0 + L_01 Sigma^T x_1 (+ Q~_0):
//   a = (sigma_s/eps) V x_0 + eps q V,  b_a = s_a A_a (slope_a(K) - slope_a(upwind)).
// Defect form (L~_00 Sigma_0^T - M_0) x_0 - L_01 Sigma^T x_1 (the same operator with
// the sigma_s/eps parts cancelled; see the 2D kernel):
//   a = eps sigma_a V x_0 + eps q V,
//   b_a = -s_a A_a (slope_a(K) - slope_a(upwind)) + A_a (T_a(K) - T_a(upwind))
// with T the outflow face value of x_0 along a (x_0 itself for LMDG; x_0 + k (x_0 -
// x_0,up) for RLMDG; zero outside the mesh).
template <typename R, int S>
__device__ __forceinline__ void raw_coef3(const double* raw, const int pos[3], const int si[3], const double A[3],
                                          bool defect, R* coef, int cstride) {
  const double x0 = raw[0];
  const double up[3] = {raw[1], raw[3], raw[5]}, upup[3] = {raw[2], raw[4], raw[6]};
  const double sl[3] = {raw[7], raw[9], raw[11]}, slu[3] = {raw[8], raw[10], raw[12]};
  const double sigtA = raw[13], absA = raw[14], scatA = raw[15], qA = raw[16];
  coef[0] = (R)sigtA;
  coef[cstride] = (R)((defect ? absA : scatA) * x0 + qA);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double ds = si[a] * A[a] * (sl[a] - slu[a]);
    double b = ds;
    if (defect) {
      double t = x0, tu = up[a];
      if (S == LMDG_SCHEME_RLMDG) {
        t = x0 + (pos[a] == 0 ? 1.0 : 0.5) * (x0 - up[a]);
        tu = pos[a] > 0 ? up[a] + (pos[a] == 1 ? 1.0 : 0.5) * (up[a] - upup[a]) : 0.0;
      }
      b = -ds + A[a] * (t - tu);
    }
    coef[(2 + a) * cstride] = (R)b;
  }
  if (S == LMDG_SCHEME_RLMDG) coef[5 * cstride] = (R)(absA * (1.0 / 3.0));
}

template <typename R, int S, int MAXW>
__global__ void __launch_bounds__(64 * MAXW) sweep3d_kernel(Sweep3Params<R> P) {
  constexpr int NOUT = Traits3<S>::NOUT;
  constexpr int NOUTP = (NOUT + 3) & ~3;  // rows of red, padded to whole lane groups
  constexpr int NF = Traits3<S>::NF;
  constexpr int NC = Traits3<S>::NC;
  constexpr int MAXC = MAXW > 4 ? 1 : kMAXC3;
  constexpr bool RLM = S == LMDG_SCHEME_RLMDG;
  extern __shared__ unsigned char smem_raw[];
  __shared__ int s_item;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int W = blockDim.x >> 6;
  const int r = lane & 15;
  const int slot = wv * 4 + (lane >> 4);
  const long long nc = P.ncell;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const long long nxy = (long long)nx * ny;
  const int lcw = P.lcw;
  const int cw = 1 << lcw;
  const int ncells = kRows << lcw;
  const int ds = P.dslots;
  const double A[3] = {P.h[1] * P.h[2], P.h[0] * P.h[2], P.h[0] * P.h[1]};
  // LDS: red [cw][W][NOUTP][16] | coef [2][NC][cw][16] | eds [cw][NF][ds] | zds [cw][16][NF][ds]
  R* red = reinterpret_cast<R*>(smem_raw);
  // one column's block of red holds W x NOUTP x 16 values plus one pad, so that the
  // reduction's reads of consecutive columns fall in different banks
  const int red_tt = W * NOUTP * kRows + 1;
  R* coef = red + (size_t)cw * red_tt;
  R* eds = coef + (size_t)2 * ncells * NC;
  R* zds = eds + (size_t)cw * NF * ds;

  for (;;) {
    if (tid == 0) s_item = (int)(atomicAdd(P.ticket, 1u) - P.ticket_base);
    __syncthreads();
    const int item = s_item;
    if (item >= P.n_items) break;
    // item = ((kz * nstrips + s) * n_rhs + rhs) * 8 + octant: both items it waits for,
    // (kz, s - 1) and (kz - 1, s), come earlier
    const int o = item & 7;
    int rest = item >> 3;
    const int rh = rest % P.n_rhs;
    rest /= P.n_rhs;
    const int s = rest % P.nstrips;
    const int kz = rest / P.nstrips;
    int si[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) si[a] = ((o >> a) & 1) ? -1 : 1;
    const double* xr = P.x ? P.x + (long long)rh * 8 * nc : nullptr;
    const double* qAr = P.qA ? P.qA + (long long)rh * nc : nullptr;
    R* const partr = P.part + (long long)rh * 8 * NOUT * nc;
    const long long ro = (long long)rh * 8 + o;
    R* const yedge = P.yedge + ro * P.yedge_ostride;                    // [nz][nstrips][nx][NF][ds]
    R* const zring = P.zbuf + ro * P.zbuf_ostride;                      // [2][ny][nx][NF][ds]
    unsigned long long* const progr = P.prog + ro * (long long)nz * P.nstrips;
    double* const psir = P.psi ? P.psi + rh * P.psi_rstride : nullptr;

    Dir3<R> d;
    {
      const double* e = P.dirs + ((long long)o * ds + slot) * kDirStride;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        d.ao[a] = (R)fabs(e[a]);
        d.aA[a] = (R)(fabs(e[a]) * A[a]);
        d.oA[a] = (R)(e[a] * A[a]);
      }
      d.w = (R)e[3];
      d.idx = (int)e[4];
    }
    const int jr = s * kRows + r;
    const bool row_ok = jr < ny;
    const int j = si[1] > 0 ? jr : ny - 1 - jr;
    const int kk = si[2] > 0 ? kz : nz - 1 - kz;
    const R ky = (jr == 0) ? R(1) : R(0.5);
    const R kzf = (kz == 0) ? R(1) : R(0.5);
    const R* zin_ring = zring + (long long)((kz + 1) & 1) * nxy * NF * ds;  // plane kz - 1
    R* const zout_ring = zring + (long long)(kz & 1) * nxy * NF * ds;

    double raw[MAXC][kNRAW3];
    auto stage_load = [&](int k) {
#pragma unroll
      for (int m = 0; m < MAXC; ++m) {
        const int e = tid + m * blockDim.x;
        const int rr = e >> lcw, tt = e & (cw - 1);
        const int c = (e < ncells) ? (k << lcw) + tt - rr : -1;
        raw_load3_impl<R>(P, xr, qAr, si, c, s * kRows + rr, kz, raw[m]);
      }
    };
    auto stage_store = [&](int k, int buf) {
#pragma unroll
      for (int m = 0; m < MAXC; ++m) {
        const int e = tid + m * blockDim.x;
        if (e < ncells) {
          const int rr = e >> lcw, tt = e & (cw - 1);
          const int pos[3] = {(k << lcw) + tt - rr, s * kRows + rr, kz};
          raw_coef3<R, S>(raw[m], pos, si, A, P.defect != 0, coef + (size_t)buf * NC * ncells + (tt << 4) + rr,
                          ncells);
        }
      }
    };

    R xin[NF], yprev[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) { xin[f] = 0; yprev[f] = 0; }

    stage_load(0);
    stage_store(0, 0);
    for (int k = 0; k < P.nchunks; ++k) {
      const int t0 = k << lcw;
      const int buf = k & 1;
      if (tid == 0 && (s > 0 || kz > 0)) {
        const int need = min(nx, t0 + cw);
        const unsigned long long target = ((P.epoch + P.wait_bias) << 32) | (unsigned long long)need;
        long long spins = 0;
        if (s > 0) {
          const unsigned long long* flag = progr + (long long)kz * P.nstrips + (s - 1);
          while (load_agent(flag) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > P.spin_limit) { atomicOr(P.err, 1); break; }
          }
        }
        if (kz > 0) {
          const unsigned long long* flag = progr + (long long)(kz - 1) * P.nstrips + s;
          while (load_agent(flag) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > P.spin_limit) { atomicOr(P.err, 1); break; }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      __syncthreads();
      {
        // y traces of strip s - 1 (same plane) for the chunk's columns
        const int ne = cw * NF * ds;
        const R* src = yedge + (((long long)kz * P.nstrips + (s - 1)) * nx + t0) * NF * ds;
        for (int e = tid; e < ne; e += blockDim.x) {
          const int c = t0 + e / (NF * ds);
          eds[e] = (s > 0 && c < nx) ? load_agent(src + e) : R(0);
        }
        // z traces of plane kz - 1 for every cell of the chunk, in batches of kZB values
        // per thread whose loads are all issued before the first is stored to LDS (one
        // load's latency per batch instead of per value)
        const int nz_e = cw * kRows * NF * ds;
        constexpr int kZB = 16;
        for (int base = 0; base < nz_e; base += kZB * (int)blockDim.x) {
          R v[kZB];
#pragma unroll
          for (int m = 0; m < kZB; ++m) {
            const int e = base + tid + m * (int)blockDim.x;
            const int fs = e % (NF * ds);
            const int cellc = e / (NF * ds);
            const int rr = cellc & 15, tt = cellc >> 4;
            const int c = t0 + tt - rr;
            const int jr2 = s * kRows + rr;
            v[m] = R(0);
            if (e < nz_e && kz > 0 && c >= 0 && c < nx && jr2 < ny) {
              const int i2 = si[0] > 0 ? c : nx - 1 - c;
              const int j2 = si[1] > 0 ? jr2 : ny - 1 - jr2;
              v[m] = load_agent(zin_ring + ((long long)j2 * nx + i2) * NF * ds + fs);
            }
          }
#pragma unroll
          for (int m = 0; m < kZB; ++m) {
            const int e = base + tid + m * (int)blockDim.x;
            if (e < nz_e) zds[e] = v[m];
          }
        }
      }
      if (k + 1 < P.nchunks) stage_load(k + 1);  // overlaps the step loop below
      lds_barrier();  // staged traces and coefficients visible; the prefetch stays in flight

      const R* cbuf = coef + (size_t)buf * NC * ncells;
      constexpr int U = kStepGroup3;
      for (int tg = 0; tg < cw; tg += U) {
        R src_g[U], sig_g[U], inv_g[U], edn_g[U][NF], zin_g[U][NF];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int tt = tg + u;
          const R* cf = cbuf + (tt << 4) + r;
          sig_g[u] = cf[0];
          src_g[u] = cf[ncells] + d.ao[0] * cf[2 * ncells] + d.ao[1] * cf[3 * ncells] + d.ao[2] * cf[4 * ncells];
          if constexpr (RLM) {
            const R kx = (t0 + tt - r == 0) ? R(1) : R(0.5);
            inv_g[u] = recip(sig_g[u] + d.aA[0] * (R(1) + kx) + d.aA[1] * (R(1) + ky) + d.aA[2] * (R(1) + kzf));
          } else {
            inv_g[u] = recip(sig_g[u] + d.aA[0] + d.aA[1] + d.aA[2]);
          }
#pragma unroll
          for (int f = 0; f < NF; ++f) {
            edn_g[u][f] = eds[((tt * NF) + f) * ds + slot];
            zin_g[u][f] = zds[(((tt << 4) + r) * NF + f) * ds + slot];
          }
        }
        R yo_g[U][NF], zo_g[U][NF], psi_g[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int tt = tg + u;
          const int c = t0 + tt - r;
          const bool act = row_ok && c >= 0 && c < nx;
          R ydn[NF];
#pragma unroll
          for (int f = 0; f < NF; ++f) {
            const R v = shr1(yprev[f]);
            ydn[f] = (r == 0) ? edn_g[u][f] : v;
            xin[f] = (c == 0) ? R(0) : xin[f];
          }
          const R* zin = zin_g[u];
          R o[NOUT], xo[NF], yo[NF], zo[NF];
          R psi;
          if constexpr (!RLM) {
            psi = (src_g[u] + d.aA[0] * xin[0] + d.aA[1] * ydn[0] + d.aA[2] * zin[0]) * inv_g[u];
            xo[0] = yo[0] = zo[0] = psi;
            o[0] = d.w * psi;
            o[1] = d.w * d.oA[0] * (xin[0] - psi);
            o[2] = d.w * d.oA[1] * (ydn[0] - psi);
            o[3] = d.w * d.oA[2] * (zin[0] - psi);
          } else {
            // traces per axis: [outflow face value, two tangential slopes, cell value];
            // tangential slopes in axis order: x carries (c_y, c_z), y (c_x, c_z), z (c_x, c_y)
            const R kx = (c == 0) ? R(1) : R(0.5);
            const R third = R(1) / R(3);
            psi = (src_g[u] + d.aA[0] * (xin[0] + kx * xin[3]) + d.aA[1] * (ydn[0] + ky * ydn[3]) +
                   d.aA[2] * (zin[0] + kzf * zin[3])) *
                  inv_g[u];
            const R cx = R(si[0]) * kx * (psi - xin[3]);
            const R cy = R(si[1]) * ky * (psi - ydn[3]);
            const R cz = R(si[2]) * kzf * (psi - zin[3]);
            xo[0] = psi + kx * (psi - xin[3]);
            xo[1] = cy;
            xo[2] = cz;
            xo[3] = psi;
            yo[0] = psi + ky * (psi - ydn[3]);
            yo[1] = cx;
            yo[2] = cz;
            yo[3] = psi;
            zo[0] = psi + kzf * (psi - zin[3]);
            zo[1] = cx;
            zo[2] = cy;
            zo[3] = psi;
            // eps sigma_a V / 3: sigma_t V / 3 of L_11 R minus (sigma_s/eps) V / 3 of M_1 P_1 R
            const R sV3 = cbuf[((tt << 4) + r) + 5 * ncells];
            o[0] = d.w * psi;
            o[1] = d.w * (d.oA[0] * (xin[0] - psi) + (sV3 + d.aA[0]) * cx +
                          third * (d.aA[1] * (cx - ydn[1]) + d.aA[2] * (cx - zin[1])));
            o[2] = d.w * (d.oA[1] * (ydn[0] - psi) + (sV3 + d.aA[1]) * cy +
                          third * (d.aA[0] * (cy - xin[1]) + d.aA[2] * (cy - zin[2])));
            o[3] = d.w * (d.oA[2] * (zin[0] - psi) + (sV3 + d.aA[2]) * cz +
                          third * (d.aA[0] * (cz - xin[2]) + d.aA[1] * (cz - ydn[2])));
            o[4] = d.w * third * (d.oA[0] * (xin[1] - cy) + d.oA[1] * (ydn[1] - cx));
            o[5] = d.w * third * (d.oA[0] * (xin[2] - cz) + d.oA[2] * (zin[1] - cx));
            o[6] = d.w * third * (d.oA[1] * (ydn[2] - cz) + d.oA[2] * (zin[2] - cy));
            o[7] = d.w * cx;
            o[8] = d.w * cy;
            o[9] = d.w * cz;
          }
          psi_g[u] = psi;
#pragma unroll
          for (int f = 0; f < NF; ++f) {
            xin[f] = xo[f];
            yprev[f] = yo[f];
            yo_g[u][f] = yo[f];
            zo_g[u][f] = zo[f];
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
            red[tt * red_tt + (wv * NOUTP + m0 + (lane >> 4)) * kRows + r] = v;
          }
        }
        // deferred stores of the group: y traces (top row), z traces (every cell), psi
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int c = t0 + tg + u - r;
          if (row_ok && c >= 0 && c < nx) {
            const int i = si[0] > 0 ? c : nx - 1 - c;
            if (r == kRows - 1 && s + 1 < P.nstrips) {
              R* e = yedge + ((((long long)kz * P.nstrips + s) * nx + c) * NF) * ds + slot;
#pragma unroll
              for (int f = 0; f < NF; ++f) store_agent(e + (long long)f * ds, yo_g[u][f]);
            }
            if (kz + 1 < nz) {
              R* e = zout_ring + (((long long)j * nx + i) * NF) * ds + slot;
#pragma unroll
              for (int f = 0; f < NF; ++f) store_agent(e + (long long)f * ds, zo_g[u][f]);
            }
            if (psir && d.idx >= 0) {
              const long long cell = (long long)kk * nxy + (long long)j * nx + i;
              psir[(long long)d.idx * nc + cell] = (double)psi_g[u];
            }
          }
        }
      }
      // publish: columns below `done` are finished by every row of this strip (also
      // their z traces, which plane kz + 1 reads, and their reads of plane kz - 1).
      // Raised before the staging and reduction below, which no other item waits for:
      // every wave waits for its own trace stores to complete before the barrier.
      const bool publish = s + 1 < P.nstrips || kz + 1 < nz;
      if (publish) __builtin_amdgcn_s_waitcnt(kWaitVmem);
      __syncthreads();
      if (tid == 0 && publish) {
        const int done = (k + 1 == P.nchunks) ? nx : min(nx, t0 + cw - (kRows - 1));
        if (done > 0) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          store_agent(progr + (long long)kz * P.nstrips + s, (P.epoch << 32) | (unsigned long long)done);
        }
      }
      if (k + 1 < P.nchunks) stage_store(k + 1, buf ^ 1);
      const int nred = (NOUT * kRows) << lcw;
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
          const int i = si[0] > 0 ? c : nx - 1 - c;
          const int jj = si[1] > 0 ? jr2 : ny - 1 - jr2;
          partr[((long long)o * NOUT + m) * nc + (long long)kk * nxy + (long long)jj * nx + i] = acc;
        }
      }
    }
    __syncthreads();
  }
}

template <typename R, int S>
size_t lds_bytes3(int cw, int W, int dslots) {
  constexpr int NOUT = Traits3<S>::NOUT;
  constexpr int NF = Traits3<S>::NF;
  constexpr int NOUTP = (NOUT + 3) & ~3;
  return ((size_t)cw * (W * NOUTP * kRows + 1) + (size_t)2 * cw * kRows * Traits3<S>::NC + (size_t)cw * NF * dslots +
          (size_t)cw * kRows * NF * dslots) *
         sizeof(R);
}

template <typename R, int S>
int launch3_typed(lmdg_handle* h, const double* x, bool use_q, double* psi, hipStream_t st, bool defect) {
  Sweep3Params<R> P;
  P.nx = (int)h->n[0];
  P.ny = (int)h->n[1];
  P.nz = (int)h->n[2];
  P.nstrips = h->nstrips;
  P.dslots = h->dslots;
  const int W = h->waves;
  // LDS per workgroup (gfx950 gives a workgroup up to 160 KB): FP64 sweeps take the
  // widest chunks that fit one workgroup per compute unit; FP32 sweeps are held to 64 KB,
  // so that two or three workgroups share a compute unit (measured faster, 128^3 S8)
  constexpr size_t kLdsBudget = sizeof(R) == 8 ? 144 * 1024 : 64 * 1024;
  int cw = 16;
  const int maxc = W > 4 ? 1 : kMAXC3;
  while (cw > kStepGroup3 && (kRows * cw > maxc * 64 * W || lds_bytes3<R, S>(cw, W, h->dslots) > kLdsBudget))
    cw >>= 1;
  if (lds_bytes3<R, S>(cw, W, h->dslots) > kLdsBudget)
    return set_error(h, LMDG_UNSUPPORTED, "direction set too large for the 3D sweep's LDS staging");
  P.cw = cw;
  P.lcw = 0;
  while ((1 << P.lcw) < cw) ++P.lcw;
  P.nchunks = (P.nx + kRows - 1 + cw - 1) / cw;
  P.n_rhs = h->n_rhs;
  P.n_items = 8 * h->nstrips * P.nz * h->n_rhs;
  for (int a = 0; a < 3; ++a) P.h[a] = h->h[a];
  P.ncell = h->ncell;
  P.dirs = h->d_dirs;
  P.x = x;
  P.sigtA = h->d_sigtA;
  P.scatA = h->d_scatA;
  P.qA = use_q ? (h->src0 ? h->src0 : h->d_qA) : nullptr;
  P.absA = h->d_absA;
  P.defect = defect ? 1 : 0;
  P.part = reinterpret_cast<R*>(h->ws.part);
  h->last_nsl = 8;
  P.yedge = reinterpret_cast<R*>(h->ws.edge);
  P.zbuf = reinterpret_cast<R*>(h->ws.zbuf);
  constexpr int NF = Traits3<S>::NF;
  P.yedge_ostride = (long long)P.nz * h->nstrips * P.nx * NF * h->dslots;
  P.zbuf_ostride = (long long)2 * P.nx * P.ny * NF * h->dslots;
  P.psi = psi;
  P.psi_rstride = (long long)h->ndir * h->ncell;
  P.prog = h->ws.prog;
  P.ticket = h->ws.ticket;
  P.err = h->ws.err;
  P.epoch = h->epoch;
  P.ticket_base = h->ticket_base;
  P.spin_limit = h->spin_limit;
  P.wait_bias = h->wait_bias;
  const int grid = std::min(P.n_items, 4 * h->n_cu);
  const size_t lds = lds_bytes3<R, S>(cw, W, h->dslots);
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
  if (W <= 4)
    hipLaunchKernelGGL((sweep3d_kernel<R, S, 4>), dim3(grid), dim3(64 * W), lds, st, P);
  else
    hipLaunchKernelGGL((sweep3d_kernel<R, S, kMaxWaves>), dim3(grid), dim3(64 * W), lds, st, P);
  if (ev_end) hipEventRecord(ev_end, st);
  h->epoch += 1;
  h->ticket_base += (unsigned)(P.n_items + grid);
  return check_hip(h, hipGetLastError(), "sweep launch");
}

}  // namespace

int launch_sweep3d(lmdg_handle* h, int scheme, int prec, const double* x, bool use_q, double* psi, hipStream_t st,
                   bool defect) {
  if (scheme == LMDG_SCHEME_STD) return set_error(h, LMDG_UNSUPPORTED, "the 3D path covers LMDG and RLMDG");
  if (prec == LMDG_PREC_FP64)
    return scheme == LMDG_SCHEME_LMDG ? launch3_typed<double, LMDG_SCHEME_LMDG>(h, x, use_q, psi, st, defect)
                                      : launch3_typed<double, LMDG_SCHEME_RLMDG>(h, x, use_q, psi, st, defect);
  return scheme == LMDG_SCHEME_LMDG ? launch3_typed<float, LMDG_SCHEME_LMDG>(h, x, use_q, psi, st, defect)
                                    : launch3_typed<float, LMDG_SCHEME_RLMDG>(h, x, use_q, psi, st, defect);
}

}  // namespace lmdg
