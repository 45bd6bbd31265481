// Internal declarations of the low-memory S_N-DG library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "lmdg.h"

namespace lmdg {

constexpr int kRows = 16;         // rows of one strip (lanes of one DPP row)
constexpr int kMaxSlots = 36;     // direction slots per quadrant (9 waves x 4; S16 has 36)
constexpr int kMaxWaves = kMaxSlots / 4;
constexpr int kDirStride = 8;     // doubles per direction-table entry
constexpr int kMaxRhs = 64;       // right-hand sides per handle

// Raw outputs of a sweep per scheme: number of per-cell reductions and of
// face-trace values handed from a cell to its downwind neighbours.
template <int S> struct SchemeTraits;
template <> struct SchemeTraits<LMDG_SCHEME_STD> { static constexpr int NOUT = 4, NF = 2; };
template <> struct SchemeTraits<LMDG_SCHEME_LMDG> { static constexpr int NOUT = 3, NF = 1; };
template <> struct SchemeTraits<LMDG_SCHEME_RLMDG> { static constexpr int NOUT = 6, NF = 3; };

// Everything the 2D sweep kernel reads; passed by value.
template <typename R>
struct SweepParams {
  int nx, ny, nstrips, cw, lcw, nchunks, dslots, n_items;  // cw = 1 << lcw steps per chunk
  int n_rhs;             // right-hand sides swept together (vectors stacked rhs-major)
  int nq;                // quadrants swept (item index runs over these only)
  int qsel[4];           // the swept quadrants
  int psi_by_slot;       // 1: psi indexed by direction slot (one quadrant), 0: by caller index
  long long psi_rstride, edge_rstride;
  double hx, hy;
  long long ncell;
  const double* dirs;    // [4][dslots][kDirStride]: ox, oy, w, index
  const double* x;       // moment vectors (n_rhs * 4 * ncell) or null
  const double* sigtA;   // (sigma_s/eps + eps sigma_a) |K|
  const double* scatA;   // (sigma_s/eps) |K|
  const double* qA;      // eps q |K| (n_rhs * ncell) or null
  const double* qS;      // source slope moments (3 * ncell, standard scheme) or null
  const double* absA;    // eps sigma_a |K|
  const double* alpha;   // inflow data [n_dir][nfaces][3] (face average, linear coefficient, midpoint) or null
  const double* qdir;    // direction-dependent source moments eps q_l |K| [n_dir][qdir_nm][ncell] or null
  int qdir_nm;           // moments per direction in qdir (4; 1 for the adjoint source)
  int nfaces;            // inflow faces per direction: n_y x faces, then n_x y faces
  int recon_y;           // 1: RLMDG reconstructs along y; 0 on slab handles
  int rflags;            // reconstruction variant: bit 0 three-cell, bit 1 suppression, bit 2 y axis
  int defect;            // 1: x enters through the defect source (see lm_source)
  R* part;               // [n_rhs][4][NOUT][ncell] per-quadrant sums
  R* edge;               // [n_rhs][4][nstrips][nx][NF][dslots] top-row traces
  double* psi;           // optional angular flux ([n_rhs][n_dir][...])
  unsigned long long* prog;   // [n_rhs][4][nstrips] progress words
  unsigned int* ticket;
  int* err;
  unsigned long long epoch;
  unsigned int ticket_base;
  long long spin_limit;  // polls of a progress word before a wait gives up
  unsigned int wait_bias;  // 0; 1 makes every wait target unreachable (failure-handling tests)
};

// Per-cell source coefficients of the 3D sweeps (sweep3d.hip coef3_kernel); passed by value.
struct Coef3Params {
  int n[3];
  int n_rhs;
  int defect;            // 1: x enters through the defect source (low-memory schemes)
  long long ncell;
  double A[3];           // face measures h_y h_z, h_x h_z, h_x h_y
  const double* x;       // moment vectors (n_rhs * 8 * ncell) or null
  const double* qA;      // eps q V (n_rhs * ncell) or null
  const double* sigtA;   // (sigma_s/eps + eps sigma_a) V
  const double* scatA;   // (sigma_s/eps) V
  const double* absA;    // eps sigma_a V
};

// Everything the 3D sweep kernel reads; passed by value.
template <typename R>
struct Sweep3Params {
  int nx, ny, nz, nstrips, nblk, dslots, n_items, n_rhs;
  double h[3];
  long long ncell;
  const double* dirs;    // [8][dslots][kDirStride]: Ox, Oy, Oz, w, index
  const R* coef;         // per-cell coefficients (coef3_kernel layout)
  R* part;               // [n_rhs][8][NOUT][ncell]
  R* xedge;              // [n_rhs][8][nz + L][nstrips][nblk][NF][dslots][16] last-column traces by period
  R* yedge;              // [n_rhs][8][nz + L][nstrips][nblk][CB][dslots][NF] top-row traces by period
  long long xedge_ostride, yedge_ostride;   // per (rhs, octant)
  double* psi;           // optional angular flux [n_rhs][n_dir][(8 moments, STD)][ncell]
  long long psi_rstride;
  unsigned long long* prog;   // [n_rhs][8][nstrips][nblk] periods completed (epoch in the high word)
  unsigned int* ticket;
  int* err;
  unsigned long long epoch;
  unsigned int ticket_base;
  long long spin_limit;
  unsigned int wait_bias;
};

struct Workspace {
  double* part = nullptr;       // 4 * 6 * ncell doubles (reused as floats)
  void* edge = nullptr;
  size_t edge_bytes = 0;
  void* zbuf = nullptr;          // 3D: per-cell sweep coefficients
  size_t zbuf_bytes = 0;          // per right-hand side
  size_t part_bytes = 0;          // per right-hand side
  size_t prog_words = 0;          // per right-hand side
  unsigned long long* prog = nullptr;
  unsigned int* ticket = nullptr;
  int* err = nullptr;
  double* vec = nullptr;        // scratch moment vectors (kScratchVecs * 4 * ncell)
};

// Two-level preconditioner (precond.hip): cell blocks K_loc^{-1}, level-0 node arrays of
// the eq-difflimPF operator, and the Cartesian multigrid levels of both parity classes.
struct PcLevel {
  int mx = 0, my = 0;
  double* S = nullptr;   // [2][9][mx my] stencils, entry (dy + 1) * 3 + dx + 1
  double* u = nullptr;   // [2][mx my]
  double* f = nullptr;
  double* r = nullptr;
};
struct Precond {
  int NX = 0, NY = 0;                      // nodes of level 0
  int kloc_scheme = -1;                    // scheme kinv was formed for
  unsigned long long kloc_mat = 0, mg_mat = 0;   // material versions they were built from
  double* kinv = nullptr;                  // [16][n_cells] row-major 4 x 4 inverses
  double* wcell = nullptr;                 // [n_cells] weights of the diagonal node pairs
  double* d0 = nullptr;                    // [NX NY] level-0 diagonal
  double* u0 = nullptr;
  double* f0 = nullptr;
  std::vector<PcLevel> lev;                // levels 1.. (last: coarsest, dense inverse)
  double* cinv = nullptr;                  // [2][m][m]
  double* cwork = nullptr;                 // [2][m][2m]
  std::vector<void*> allocs;
  size_t bytes = 0;
};

}  // namespace lmdg

struct lmdg_handle {
  int dim = 2;
  bool slab = false;               // 2D handle standing for a slab problem (lmdg_create with dim 1)
  int64_t n[3] = {0, 0, 1};
  double len[3] = {1, 1, 1}, h[3] = {1, 1, 1}, area = 1;   // area: cell measure (|K| in 2D, V in 3D)
  long long ncell = 0;
  int n_rhs = 1;                   // right-hand sides (sources) of the handle
  int rhs_cap = 1;                 // right-hand sides the workspaces are sized for
  int np = 4;
  int ndir = 0;
  std::vector<double> omega, w;
  int dslots = 4, waves = 1, nstrips = 0;
  std::vector<int> slot_dir;      // [4][dslots], -1 = padding
  double* d_dirs = nullptr;
  double cplus[3] = {0, 0, 0}, cminus[3] = {0, 0, 0};
  int noct = 4;                    // quadrants (2D) or octants (3D)
  // per-quadrant (octant) sums of w and w |Omega_a| (used by the defect combine)
  double qw[8] = {0}, qax[8] = {0}, qay[8] = {0}, qaz[8] = {0};
  bool have_mat = false;
  double* d_sigtA = nullptr;
  double* d_scatA = nullptr;
  double* d_absA = nullptr;        // eps sigma_a |K|
  double* d_qA = nullptr;
  double* d_epsA = nullptr;        // eps |K| (gradients)
  std::vector<double> h_eps;       // host copy of eps (source scaling)
  // source used by sweeps with use_q: src0 replaces eps q |K| when set, src1 adds
  // slope moments (standard scheme); both null outside the adjoint solve
  const double* src0 = nullptr;
  const double* src1 = nullptr;
  // the handle's own source data beyond per-cell constants (2D, one right-hand side):
  // d_qS   source slope moments eps q_r |K|, r = 1..3, of an isotropic source (STD sweeps)
  // d_qdir direction-dependent source moments eps q_{l,r} |K| [n_dir][4][ncell]
  // d_alpha inflow data [n_dir][n_x + n_y][3] (see SweepParams::alpha)
  // d_sq1  sum_l w_l of the source slope moments (3 x ncell), subtracted from the slope
  //        rows of the low-memory right-hand sides
  // d_sqa  the part of the inflow terms of the LMDG slope rows that the sweep's ghost
  //        traces do not carry (3 x ncell), subtracted likewise
  double* d_qS = nullptr;
  double* d_qdir = nullptr;
  double* d_alpha = nullptr;
  double* d_sq1 = nullptr;
  double* d_sqa = nullptr;
  int last_nsl = 4;                // partial slices written by the last sweep launch
  int recon_flags = 0;             // RLMDG reconstruction variant (lmdg_set_reconstruction)
  // adjoint of RLMDG (inside lmdg_adjoint_solve): sweeps, right-hand sides, recovery and
  // K x take the adjoint system; d_adjsrc holds its per-direction source [n_dir][ncell]
  bool adj_rlm = false;
  const double* adj_det = nullptr;
  double* d_adjsrc = nullptr;
  // directions: index of -Omega_l; per quadrant and slot the weight and the slot of
  // -Omega_l in the opposite quadrant (adjoint gradients)
  std::vector<int> neg_dir;
  double* d_adjpairs = nullptr;    // [4][dslots][2]
  double* d_psi_f = nullptr;       // one quadrant's angular fluxes (adjoint gradients)
  double* d_psi_a = nullptr;
  size_t psi_doubles = 0;
  double* d_cvec = nullptr;        // adjoint vectors: c, x (forward), phi, Lambda, x (adjoint), bilinear sums
  lmdg::Workspace ws;
  unsigned long long epoch = 1;
  unsigned int ticket_base = 0;
  long long spin_limit = 1ll << 25;  // polls per wait (lmdg_set_wait_limit)
  unsigned int wait_bias = 0;
  int device = 0;
  int n_cu = 256;
  std::string last_error;
  // sweep-kernel timing (lmdg_profile)
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  // Krylov workspace (grown on demand)
  double* d_krylov = nullptr;
  size_t krylov_doubles = 0;
  double* d_small = nullptr;       // device scratch for dot products
  double* h_small = nullptr;       // pinned host mirror
  size_t small_doubles = 0;
  int augment = 0;                 // LGMRES: stored corrections searched per restart cycle
  double ir_inner = 1e-3;          // mode MIXED: residual reduction asked of each inner FP32 solve
  unsigned long long mat_version = 0;   // bumped by lmdg_set_materials
  int pc_kind = 0;                 // LMDG_PRECOND_* used by the solves
  int pc_cycles = 1;               // V-cycles per application of the two-level preconditioner
  lmdg::Precond* pc = nullptr;
};

namespace lmdg {

constexpr int kScratchVecs = 4;

// Slices of the sweep partials per right-hand side, each [NOUT][n_cells]: FP64 2D sweeps
// with at most one work item (quadrant, strip, source) per compute unit and at most 24
// per-wave values per cell and quadrant (waves x NOUT; S8 RLMDG 18, S12 LMDG 18) write
// one slice per (quadrant, wave), measured faster there; other 2D sweeps (S16 RLMDG 54
// measured slower) one per quadrant, 3D sweeps one per octant.  The sweep launch and the
// kernels that read the partials take the same decision from the handle's current state.
inline int part_slices_max(const lmdg_handle* h) {
  if (h->dim == 3) return 8;
  return h->waves * 3 <= 24 ? 4 * h->waves : 4;  // 3 = the fewest outputs of a scheme (LMDG)
}
inline int part_slices(const lmdg_handle* h, int scheme, int prec) {
  if (h->dim == 3) return 8;
  const int nout = scheme == LMDG_SCHEME_STD ? 4 : (scheme == LMDG_SCHEME_LMDG ? 3 : 6);
  const bool direct = prec == LMDG_PREC_FP64 && 4LL * h->nstrips * h->n_rhs <= h->n_cu && h->waves * nout <= 24;
  return direct ? 4 * h->waves : 4;
}

// launchers (sweep2d.hip / ops.hip)
// p1r: the sweep also produces the P_1 R rows of RLMDG (false when the combine that
// follows reads only the operator rows: operator applications and right-hand sides)
int launch_sweep(lmdg_handle* h, int scheme, int prec, const double* x, bool use_q,
                 double* psi, hipStream_t st, bool defect = false, int qmask = 0xF,
                 bool psi_by_slot = false, bool p1r = true);
int launch_sweep3d(lmdg_handle* h, int scheme, int prec, const double* x, bool use_q, double* psi,
                   hipStream_t st, bool defect, bool p1r);
// workspace of the 3D sweeps per right-hand side (sweep3d.hip)
size_t sweep3d_edge_bytes(const lmdg_handle* h);
size_t sweep3d_coef_bytes(const lmdg_handle* h);
size_t sweep3d_prog_words(const lmdg_handle* h);
void launch_combine(lmdg_handle* h, int scheme, int prec, int mode, const double* x,
                    double* out, hipStream_t st);
void launch_sum_quadrants(lmdg_handle* h, int scheme, int prec, double* out, hipStream_t st);
void launch_combine3(lmdg_handle* h, int scheme, int prec, int mode, const double* x, double* out,
                     hipStream_t st);
void launch_sum_octants(lmdg_handle* h, int scheme, int prec, double* out, hipStream_t st);
void launch_b11_3d(lmdg_handle* h, const double* x, double* y, hipStream_t st);
void launch_b11(lmdg_handle* h, const double* x, double* y, hipStream_t st);
void launch_adj_rlm_source(lmdg_handle* h, const double* x, const double* det, hipStream_t st);
void launch_grad_accumulate(lmdg_handle* h, int quadrant, int npsi, double* bil, hipStream_t st);
void launch_gradients(lmdg_handle* h, int npsi, const double* bil, const double* phi, const double* Lam, double* gs,
                      double* ga, double* gq, hipStream_t st);

// kApplyDefect: K x from a sweep run with the defect source (same operator).
enum CombineMode { kApply = 0, kRhs = 1, kRecover = 2, kApplyDefect = 3 };

// GMRES vector kernels (ops.hip).  Vectors of nr right-hand sides are stacked in
// segments of length n; dot products and coefficients are indexed [v * nr + segment].
void vec_dots(const double* V, long long ld, int nvec, const double* w, long long n,
              double* partial, double* out, hipStream_t st, int nr = 1);
void vec_axpy_multi(double* w, const double* V, long long ld, int nvec, const double* coef,
                    double sign, long long n, hipStream_t st, int nr = 1);
void vec_scale_seg(double* y, const double* x, const double* scale, long long n, int nr, hipStream_t st);
// FP32 Krylov basis (the inner solves of mode MIXED): products and sums in FP64
void vec_dots(const float* V, long long ld, int nvec, const double* w, long long n, double* partial, double* out,
              hipStream_t st, int nr = 1);
void vec_axpy_multi(double* w, const float* V, long long ld, int nvec, const double* coef, double sign,
                    long long n, hipStream_t st, int nr = 1);
void vec_scale_seg(float* y, const double* x, const double* scale, long long n, int nr, hipStream_t st);
void vec_widen(double* y, const float* x, long long n, hipStream_t st);
void vec_axpby(double* y, double a, const double* x, double b, long long n, hipStream_t st);
void vec_copy(double* y, const double* x, long long n, hipStream_t st);
void vec_fill(double* y, double v, long long n, hipStream_t st);
int dots_partials();

// two-level preconditioner (precond.hip)
bool pc_supported(const lmdg_handle* h, int scheme, std::string* why);
int pc_prepare(lmdg_handle* h, int scheme, hipStream_t st);
int pc_apply(lmdg_handle* h, int scheme, const double* r, double* z, hipStream_t st);
void pc_free(lmdg_handle* h);
size_t pc_bytes(const lmdg_handle* h);

int set_error(lmdg_handle* h, int status, const std::string& msg);
int check_hip(lmdg_handle* h, hipError_t e, const char* what);

}  // namespace lmdg
