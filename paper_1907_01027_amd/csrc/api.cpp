// Host side of the C ABI: quadrature generation, handle set-up, validation, and the
// FP64 GMRES / iterative-refinement drivers around the device kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

using lmdg::check_hip;
using lmdg::set_error;

namespace lmdg {

int set_error(lmdg_handle* h, int status, const std::string& msg) {
  if (h) h->last_error = msg;
  return status;
}

int check_hip(lmdg_handle* h, hipError_t e, const char* what) {
  if (e == hipSuccess) return LMDG_OK;
  return set_error(h, LMDG_HIP_ERROR, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

// ------------------------------------------------------------------ quadrature
// Small dense solve with partial pivoting (n <= 16), in place; returns false if singular.
bool dense_solve(std::vector<double>& A, std::vector<double>& b, int n) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[i * n + k]) > std::fabs(A[piv * n + k])) piv = i;
    if (A[piv * n + k] == 0.0) return false;
    if (piv != k) {
      for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[piv * n + j]);
      std::swap(b[k], b[piv]);
    }
    for (int i = k + 1; i < n; ++i) {
      const double f = A[i * n + k] / A[k * n + k];
      for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
      b[i] -= f * b[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    double acc = b[k];
    for (int j = k + 1; j < n; ++j) acc -= A[k * n + j] * b[j];
    b[k] = acc / A[k * n + k];
  }
  return true;
}

struct Octant {
  std::vector<double> mu;           // levels
  std::vector<int> pi, pj, pk;      // level indices of the points
  std::vector<int> cls;             // class of each point
  int ncls = 0;
};

Octant octant(int order, double mu1) {
  Octant o;
  const int nl = order / 2;
  const double step = 2.0 * (1.0 - 3.0 * mu1 * mu1) / (order - 2);
  for (int i = 0; i < nl; ++i) o.mu.push_back(std::sqrt(mu1 * mu1 + step * i));
  std::vector<std::vector<int>> keys;
  for (int i = 1; i <= nl; ++i)
    for (int j = 1; j <= nl; ++j) {
      const int k = nl + 2 - i - j;
      if (k < 1 || k > nl) continue;
      std::vector<int> key = {i, j, k};
      std::sort(key.begin(), key.end());
      int c = (int)(std::find(keys.begin(), keys.end(), key) - keys.begin());
      if (c == (int)keys.size()) keys.push_back(key);
      o.pi.push_back(i - 1);
      o.pj.push_back(j - 1);
      o.pk.push_back(k - 1);
      o.cls.push_back(c);
    }
  // classes numbered in sorted order of their index triples
  std::vector<int> perm(keys.size());
  for (size_t c = 0; c < keys.size(); ++c) perm[c] = (int)c;
  std::sort(perm.begin(), perm.end(), [&](int a, int b) { return keys[a] < keys[b]; });
  std::vector<int> rank(keys.size());
  for (size_t c = 0; c < perm.size(); ++c) rank[perm[c]] = (int)c;
  for (auto& c : o.cls) c = rank[c];
  o.ncls = (int)keys.size();
  return o;
}

// Even moments imposed on the class weights, and the one used to pick mu_1.
void moments(int order, int ncls, std::vector<int>& imposed, int& check) {
  imposed = {0};
  const int top = (order == 16) ? 7 : ncls;  // N = 16: 8 classes, rank-7 system
  for (int m = 2; m <= top; ++m) imposed.push_back(m);
  check = std::max(imposed.back() + 1, 2);
}

// Minimum-norm class weights w = A^T (A A^T)^{-1} b of sum_octant w mu_z^(2m) = 1/(8(2m+1)).
bool class_weights(int order, double mu1, std::vector<double>& wc, Octant& o) {
  o = octant(order, mu1);
  std::vector<int> imp;
  int check;
  moments(order, o.ncls, imp, check);
  const int ne = (int)imp.size(), nc = o.ncls;
  std::vector<double> A(ne * nc, 0.0), b(ne);
  for (size_t p = 0; p < o.cls.size(); ++p)
    for (int e = 0; e < ne; ++e) A[e * nc + o.cls[p]] += std::pow(o.mu[o.pk[p]], 2 * imp[e]);
  for (int e = 0; e < ne; ++e) b[e] = 1.0 / (8.0 * (2 * imp[e] + 1));
  std::vector<double> G(ne * ne, 0.0);
  for (int a = 0; a < ne; ++a)
    for (int c = 0; c < ne; ++c)
      for (int k = 0; k < nc; ++k) G[a * ne + c] += A[a * nc + k] * A[c * nc + k];
  if (!dense_solve(G, b, ne)) return false;
  wc.assign(nc, 0.0);
  for (int k = 0; k < nc; ++k)
    for (int e = 0; e < ne; ++e) wc[k] += A[e * nc + k] * b[e];
  return true;
}

double extra_moment_residual(int order, double mu1) {
  std::vector<double> wc;
  Octant o;
  if (!class_weights(order, mu1, wc, o)) return NAN;
  std::vector<int> imp;
  int check;
  moments(order, o.ncls, imp, check);
  double acc = 0;
  for (size_t p = 0; p < o.cls.size(); ++p) acc += wc[o.cls[p]] * std::pow(o.mu[o.pk[p]], 2 * check);
  return 8.0 * acc - 1.0 / (2 * check + 1);
}

double mu1_guess(int order) {
  switch (order) {
    case 4: return 0.3500212;
    case 6: return 0.2666355;
    case 8: return 0.2182179;
    case 12: return 0.1672126;
    case 16: return 0.1389568;
    default: return 0.0;
  }
}

}  // namespace
}  // namespace lmdg

extern "C" {

const char* lmdg_status_string(int status) {
  switch (status) {
    case LMDG_OK: return "ok";
    case LMDG_INVALID_ARG: return "invalid argument";
    case LMDG_NOT_CONVERGED: return "not converged";
    case LMDG_NONFINITE: return "non-finite value";
    case LMDG_HIP_ERROR: return "HIP runtime error";
    case LMDG_UNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
  }
}

const char* lmdg_last_error(const lmdg_t* h) {
  if (!h) return "no handle";
  return h->last_error.c_str();
}

int lmdg_quadrature_level_symmetric(int dim, int order, int capacity, int* n_dir, double* omega, double* w) {
  using namespace lmdg;
  if ((dim != 2 && dim != 3) || mu1_guess(order) == 0.0 || !n_dir || !omega || !w) return LMDG_INVALID_ARG;
  const int count = dim == 2 ? order * (order + 2) / 2 : order * (order + 2);
  if (capacity < count) return LMDG_INVALID_ARG;
  // bisection on the first non-imposed even moment, bracket +-10% around the table value
  double lo = 0.9 * mu1_guess(order), hi = 1.1 * mu1_guess(order);
  double flo = extra_moment_residual(order, lo), fhi = extra_moment_residual(order, hi);
  if (!(flo * fhi < 0)) return LMDG_INVALID_ARG;
  for (int it = 0; it < 200 && hi - lo > 1e-17; ++it) {
    const double mid = 0.5 * (lo + hi);
    const double fm = extra_moment_residual(order, mid);
    if (fm == 0.0) { lo = hi = mid; break; }
    if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { hi = mid; }
  }
  const double mu1 = 0.5 * (lo + hi);
  std::vector<double> wc;
  Octant o;
  if (!class_weights(order, mu1, wc, o)) return LMDG_INVALID_ARG;
  for (double v : wc)
    if (!(v > 0)) return LMDG_INVALID_ARG;
  const int npts = (int)o.cls.size();
  const int noct = 1 << dim;
  double total = 0;
  int k = 0;
  for (int oc = 0; oc < noct; ++oc)
    for (int p = 0; p < npts; ++p) {
      const double pt[3] = {o.mu[o.pi[p]], o.mu[o.pj[p]], o.mu[o.pk[p]]};
      for (int a = 0; a < dim; ++a) omega[k * dim + a] = ((oc >> a) & 1) ? -pt[a] : pt[a];
      w[k] = wc[o.cls[p]];
      total += w[k];
      ++k;
    }
  for (int i = 0; i < k; ++i) w[i] /= total;
  *n_dir = k;
  return LMDG_OK;
}

// Grow the per-right-hand-side workspaces (partials, strip edges, 3D coefficients,
// progress words, scratch vectors, sources) to n_rhs right-hand sides.
static int ensure_rhs_capacity(lmdg_t* h, int n_rhs) {
  using namespace lmdg;
  if (n_rhs <= h->rhs_cap) return LMDG_OK;
  hipDeviceSynchronize();
  const long long nc = h->ncell;
  void* olds[] = {h->ws.part, h->ws.edge, h->ws.zbuf, h->ws.prog, h->ws.vec, h->d_qA};
  for (void* p : olds)
    if (p) hipFree(p);
  h->ws.part = nullptr;
  h->ws.edge = nullptr;
  h->ws.zbuf = nullptr;
  h->ws.prog = nullptr;
  h->ws.vec = nullptr;
  h->d_qA = nullptr;
  h->rhs_cap = 0;
  const size_t nr = (size_t)n_rhs;
  int rc = check_hip(h, hipMalloc((void**)&h->ws.part, h->ws.part_bytes * nr), "hipMalloc");
  if (rc == LMDG_OK) rc = check_hip(h, hipMalloc(&h->ws.edge, std::max<size_t>(h->ws.edge_bytes * nr, 8)), "hipMalloc");
  if (rc == LMDG_OK && h->ws.zbuf_bytes)
    rc = check_hip(h, hipMalloc(&h->ws.zbuf, h->ws.zbuf_bytes * nr), "hipMalloc");
  if (rc == LMDG_OK)
    rc = check_hip(h, hipMalloc((void**)&h->ws.prog, h->ws.prog_words * nr * sizeof(unsigned long long)), "hipMalloc");
  if (rc == LMDG_OK)
    rc = check_hip(h, hipMalloc((void**)&h->ws.vec, (size_t)kScratchVecs * h->np * nc * nr * sizeof(double)),
                   "hipMalloc");
  if (rc == LMDG_OK) rc = check_hip(h, hipMalloc((void**)&h->d_qA, (size_t)nc * nr * sizeof(double)), "hipMalloc");
  if (rc == LMDG_OK)
    rc = check_hip(h, hipMemset(h->ws.prog, 0, h->ws.prog_words * nr * sizeof(unsigned long long)), "clear flags");
  if (rc == LMDG_OK) rc = check_hip(h, hipDeviceSynchronize(), "workspaces");
  if (rc == LMDG_OK) h->rhs_cap = n_rhs;
  return rc;
}

// Body of lmdg_create for 2D and 3D handles.  slab: a 2D handle standing for the slab
// problem (one row of cells, every Omega_y = 0), where the y components are exempt from
// the nonzero-component and second-moment checks.
static int create_impl(int dim, const int64_t* n, const double* length, int n_dir, const double* omega,
                       const double* w, lmdg_t** out, bool slab) {
  using namespace lmdg;
  long long ncell = 1;
  for (int a = 0; a < dim; ++a) {
    if (n[a] < 1 || n[a] > (1 << 20) || !(length[a] > 0) || !std::isfinite(length[a])) return LMDG_INVALID_ARG;
    ncell *= n[a];
  }
  if (n_dir < 1 || ncell > (1ll << 31)) return LMDG_INVALID_ARG;
  // eq-polyquad (i)-(iii), positive weights, no zero component
  double s0 = 0, s1[3] = {0, 0, 0}, s2[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int l = 0; l < n_dir; ++l) {
    if (!(w[l] > 0) || !std::isfinite(w[l])) return LMDG_INVALID_ARG;
    for (int a = 0; a < dim; ++a)
      if (!std::isfinite(omega[dim * l + a]) || (omega[dim * l + a] == 0.0 && !(slab && a == 1)))
        return LMDG_INVALID_ARG;
    s0 += w[l];
    for (int a = 0; a < dim; ++a) {
      s1[a] += w[l] * omega[dim * l + a];
      for (int b = 0; b < dim; ++b) s2[a][b] += w[l] * omega[dim * l + a] * omega[dim * l + b];
    }
  }
  const double tq = 1e-12;
  if (std::fabs(s0 - 1) > tq) return LMDG_INVALID_ARG;
  for (int a = 0; a < dim; ++a) {
    if (std::fabs(s1[a]) > tq) return LMDG_INVALID_ARG;
    for (int b = 0; b < dim; ++b)
      if (std::fabs(s2[a][b] - (a == b && !(slab && a == 1) ? 1.0 / 3.0 : 0.0)) > tq) return LMDG_INVALID_ARG;
  }
  lmdg_handle* h = new (std::nothrow) lmdg_handle();
  if (!h) return LMDG_HIP_ERROR;
  h->dim = dim;
  h->slab = slab;
  h->np = dim == 2 ? 4 : 8;
  h->noct = 1 << dim;
  h->area = 1.0;
  for (int a = 0; a < dim; ++a) {
    h->n[a] = n[a];
    h->len[a] = length[a];
    h->h[a] = length[a] / (double)n[a];
    h->area *= h->h[a];
  }
  h->ncell = ncell;
  h->ndir = n_dir;
  h->omega.assign(omega, omega + dim * n_dir);
  h->w.assign(w, w + n_dir);
  // quadrant / octant q: bit a set when Omega_a < 0
  auto octant = [&](int l) {
    int q = 0;
    for (int a = 0; a < dim; ++a) q |= (omega[dim * l + a] < 0 ? 1 : 0) << a;
    return q;
  };
  std::vector<int> byq[8];
  for (int l = 0; l < n_dir; ++l) byq[octant(l)].push_back(l);
  size_t dmax = 1;
  for (int q = 0; q < h->noct; ++q) dmax = std::max(dmax, byq[q].size());
  if (dmax > (size_t)kMaxSlots) {
    delete h;
    return LMDG_INVALID_ARG;
  }
  h->dslots = (int)((dmax + 3) / 4 * 4);
  h->waves = h->dslots / 4;
  h->nstrips = (int)((n[1] + kRows - 1) / kRows);
  // direction table: 2D entries (Ox, Oy, w, index), 3D entries (Ox, Oy, Oz, w, index)
  std::vector<double> tab((size_t)h->noct * h->dslots * kDirStride, 0.0);
  h->slot_dir.assign((size_t)h->noct * h->dslots, -1);
  for (int q = 0; q < h->noct; ++q) {
    // padding slots copy a real direction of the quadrant (or the quadrant's sign
    // pattern) with zero weight, so they compute finite values and contribute nothing
    double pad[3];
    for (int a = 0; a < dim; ++a) pad[a] = ((q >> a) & 1) ? -0.5 : 0.5;
    if (!byq[q].empty())
      for (int a = 0; a < dim; ++a) pad[a] = omega[dim * byq[q][0] + a];
    for (int sl = 0; sl < h->dslots; ++sl) {
      double* e = &tab[((size_t)q * h->dslots + sl) * kDirStride];
      const bool real = sl < (int)byq[q].size();
      const int l = real ? byq[q][sl] : -1;
      for (int a = 0; a < dim; ++a) e[a] = real ? omega[dim * l + a] : pad[a];
      e[dim] = real ? w[l] : 0.0;
      e[dim + 1] = l;
      h->slot_dir[(size_t)q * h->dslots + sl] = l;
    }
  }
  for (int l = 0; l < n_dir; ++l) {
    const int q = octant(l);
    h->qw[q] += w[l];
    double* qa[3] = {h->qax, h->qay, h->qaz};
    for (int a = 0; a < dim; ++a) {
      const double o = omega[dim * l + a];
      if (o > 0) h->cplus[a] += w[l] * o; else h->cminus[a] += w[l] * (-o);
      qa[a][q] += w[l] * std::fabs(o);
    }
  }
  // -Omega_l for every l (central symmetry), used by the adjoint; -1 when absent
  h->neg_dir.assign(n_dir, -1);
  for (int l = 0; l < n_dir; ++l)
    for (int k = 0; k < n_dir; ++k) {
      bool match = std::fabs(w[k] - w[l]) <= 1e-12 * w[l];
      for (int a = 0; a < dim; ++a) match = match && std::fabs(omega[dim * k + a] + omega[dim * l + a]) <= 1e-12;
      if (match) {
        h->neg_dir[l] = k;
        break;
      }
    }
  // per-right-hand-side workspace sizes
  const long long nc = h->ncell;
  if (dim == 2) {
    h->ws.part_bytes = (size_t)lmdg::part_slices_max(h) * 6 * nc * sizeof(double);
    // up to four trace values per direction slot (RLMDG with a reconstruction variant)
    h->ws.edge_bytes = (size_t)4 * h->nstrips * n[0] * 4 * h->dslots * sizeof(double);
    h->ws.zbuf_bytes = 0;
    h->ws.prog_words = (size_t)4 * h->nstrips;
  } else {
    h->ws.part_bytes = (size_t)8 * 10 * nc * sizeof(double);
    h->ws.edge_bytes = lmdg::sweep3d_edge_bytes(h);
    h->ws.zbuf_bytes = lmdg::sweep3d_coef_bytes(h);
    h->ws.prog_words = lmdg::sweep3d_prog_words(h);
  }
  int dev = 0;
  hipGetDevice(&dev);
  h->device = dev;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
    h->n_cu = prop.multiProcessorCount;
  h->rhs_cap = 0;
  int st = check_hip(h, hipMalloc((void**)&h->d_dirs, tab.size() * sizeof(double)), "hipMalloc");
  if (st == LMDG_OK) st = check_hip(h, hipMalloc((void**)&h->ws.ticket, sizeof(unsigned int)), "hipMalloc");
  if (st == LMDG_OK) st = check_hip(h, hipMalloc((void**)&h->ws.err, sizeof(int)), "hipMalloc");
  const size_t npairs = (size_t)h->noct * h->dslots * 2;
  if (st == LMDG_OK) st = check_hip(h, hipMalloc((void**)&h->d_adjpairs, npairs * sizeof(double)), "hipMalloc");
  if (st == LMDG_OK) st = ensure_rhs_capacity(h, 1);
  // per quadrant and slot: weight and the slot of -Omega in the opposite quadrant
  std::vector<double> pairs(npairs, 0.0);
  const int qmask_all = h->noct - 1;
  for (int q = 0; q < h->noct; ++q)
    for (int k = 0; k < h->dslots; ++k) {
      const int l = h->slot_dir[(size_t)q * h->dslots + k];
      if (l < 0 || h->neg_dir[l] < 0) continue;
      const int qo = q ^ qmask_all;
      for (int k2 = 0; k2 < h->dslots; ++k2)
        if (h->slot_dir[(size_t)qo * h->dslots + k2] == h->neg_dir[l]) {
          pairs[((size_t)q * h->dslots + k) * 2] = w[l];
          pairs[((size_t)q * h->dslots + k) * 2 + 1] = k2;
        }
    }
  if (st == LMDG_OK) st = check_hip(h, hipMemcpy(h->d_dirs, tab.data(), tab.size() * sizeof(double),
                                                 hipMemcpyHostToDevice), "copy directions");
  if (st == LMDG_OK) st = check_hip(h, hipMemcpy(h->d_adjpairs, pairs.data(), pairs.size() * sizeof(double),
                                                 hipMemcpyHostToDevice), "copy direction pairs");
  if (st == LMDG_OK) st = check_hip(h, hipMemset(h->ws.ticket, 0, sizeof(unsigned int)), "clear ticket");
  if (st == LMDG_OK) st = check_hip(h, hipMemset(h->ws.err, 0, sizeof(int)), "clear error flag");
  if (st == LMDG_OK) st = check_hip(h, hipDeviceSynchronize(), "create");
  if (st != LMDG_OK) {
    lmdg_destroy(h);
    return st;
  }
  *out = h;
  return LMDG_OK;
}

int lmdg_create(int dim, const int64_t* n, const double* length, int n_dir, const double* omega,
                const double* w, lmdg_t** out) {
  if (!out || !n || !length || !omega || !w) return LMDG_INVALID_ARG;
  *out = nullptr;
  if (dim == 2 || dim == 3) return create_impl(dim, n, length, n_dir, omega, w, out, false);
  if (dim != 1) return LMDG_UNSUPPORTED;
  // Slab geometry (eq-1d): the 2D problem on n[0] x 1 cells of [0, length[0]] x [0, 1]
  // with directions (mu, 0).  With Omega_y = 0 no y face carries flux, so the 1 and xi
  // moments of its solution are those of the slab scheme; the 1D rule must satisfy
  // sum w = 1, sum w mu = 0, sum w mu^2 = 1/3 (the 2D second-moment check is replaced).
  if (n_dir < 1 || n_dir > (1 << 20)) return LMDG_INVALID_ARG;
  std::vector<double> om2(2 * (size_t)n_dir);
  for (int l = 0; l < n_dir; ++l) {
    om2[2 * l] = omega[l];
    om2[2 * l + 1] = 0.0;
  }
  double m2 = 0;
  for (int l = 0; l < n_dir; ++l) m2 += w[l] * omega[l] * omega[l];
  if (!(std::fabs(m2 - 1.0 / 3.0) <= 1e-12)) return LMDG_INVALID_ARG;
  const int64_t n2[2] = {n[0], 1};
  const double len2[2] = {length[0], 1.0};
  return create_impl(2, n2, len2, n_dir, om2.data(), w, out, true);
}

void lmdg_destroy(lmdg_t* h) {
  if (!h) return;
  hipDeviceSynchronize();
  void* ptrs[] = {h->d_dirs, h->d_sigtA, h->d_scatA, h->d_absA, h->d_qA, h->ws.part, h->ws.edge, h->ws.zbuf,
                  h->ws.prog, h->ws.ticket, h->ws.err, h->ws.vec, h->d_krylov, h->d_small,
                  h->d_epsA, h->d_adjpairs, h->d_psi_f, h->d_psi_a, h->d_cvec, h->d_qS, h->d_qdir,
                  h->d_alpha, h->d_sq1, h->d_sqa, h->d_adjsrc};
  for (void* p : ptrs)
    if (p) hipFree(p);
  if (h->h_small) hipHostFree(h->h_small);
  lmdg::pc_free(h);
  for (hipEvent_t e : h->ev_pool) hipEventDestroy(e);
  delete h;
}

// Free the handle's source data beyond per-cell constants (moments, direction-dependent
// sources and their right-hand-side corrections); keep_alpha keeps the inflow data.
static void clear_source_data(lmdg_t* h, bool keep_alpha) {
  double** ptrs[] = {&h->d_qS, &h->d_qdir, &h->d_sq1, &h->d_alpha, &h->d_sqa};
  for (int k = 0; k < 5; ++k) {
    if (keep_alpha && k >= 3) break;
    if (*ptrs[k]) hipFree(*ptrs[k]);
    *ptrs[k] = nullptr;
  }
}

static int upload(lmdg_t* h, double** dst, const std::vector<double>& v, hipStream_t st) {
  int rc = check_hip(h, hipMalloc((void**)dst, v.size() * sizeof(double)), "hipMalloc source data");
  if (rc == LMDG_OK)
    rc = check_hip(h, hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, st),
                   "write source data");
  if (rc == LMDG_OK) rc = check_hip(h, hipStreamSynchronize(st), "write source data");
  return rc;
}

// Inflow data (eq-main, Gamma^-) of a 2D or slab handle, read from the caller's device
// array: 2D [n_dir][n_1 + n_0][3], slab [n_dir].  Stores the 2D layout and the part of
// the LMDG slope-row inflow terms that the ghost face averages do not carry: per
// inflow face the boundary term -int_F alpha Omega.nu v of a slope test function v
// (Q_alpha of eq-Ljk) with alpha = a0 + a1 t on the face (t the cell coordinate along
// the face) is, for an x face, -Ox h_y a0 (xi row), |Ox| h_y a1 / 3 (eta row),
// -Ox h_y a1 / 3 (xi eta row); the ghost trace a0 of the LMDG sweep gives the xi row.
static int set_alpha(lmdg_t* h, const double* alpha, hipStream_t st) {
  const int nx = (int)h->n[0], ny = (int)h->n[1], nf = nx + ny;
  const long long nc = h->ncell;
  const size_t nin = h->slab ? (size_t)h->ndir : (size_t)h->ndir * nf * 3;
  std::vector<double> a(nin);
  int rc = check_hip(h, hipMemcpyAsync(a.data(), alpha, nin * sizeof(double), hipMemcpyDeviceToHost, st),
                     "read alpha");
  if (rc == LMDG_OK) rc = check_hip(h, hipStreamSynchronize(st), "read alpha");
  if (rc != LMDG_OK) return rc;
  for (double v : a)
    if (!std::isfinite(v)) return set_error(h, LMDG_NONFINITE, "non-finite inflow value");
  std::vector<double> full((size_t)h->ndir * nf * 3, 0.0);
  if (h->slab) {
    // the x-inflow face of the single row carries the slab datum; y faces carry no flux
    for (int l = 0; l < h->ndir; ++l) {
      full[((size_t)l * nf) * 3 + 0] = a[l];
      full[((size_t)l * nf) * 3 + 2] = a[l];
    }
  } else {
    full = a;
  }
  std::vector<double> sqa(3 * (size_t)nc, 0.0);
  const double hx = h->h[0], hy = h->h[1];
  for (int l = 0; l < h->ndir; ++l) {
    const double ox = h->omega[2 * l], oy = h->omega[2 * l + 1], w = h->w[l];
    const int i0 = ox < 0 ? nx - 1 : 0, j0 = oy < 0 ? ny - 1 : 0;  // inflow column and row
    for (int j = 0; j < ny; ++j) {
      const double a1 = full[((size_t)l * nf + j) * 3 + 1];
      const long long p = (long long)j * nx + i0;
      sqa[nc + p] += w * std::fabs(ox) * hy * a1 / 3.0;
      sqa[2 * nc + p] += -w * ox * hy * a1 / 3.0;
    }
    for (int i = 0; i < nx; ++i) {
      const double b1 = full[((size_t)l * nf + ny + i) * 3 + 1];
      const long long p = (long long)j0 * nx + i;
      sqa[p] += w * std::fabs(oy) * hx * b1 / 3.0;
      sqa[2 * nc + p] += -w * oy * hx * b1 / 3.0;
    }
  }
  rc = upload(h, &h->d_alpha, full, st);
  if (rc == LMDG_OK) rc = upload(h, &h->d_sqa, sqa, st);
  return rc;
}

int lmdg_set_materials(lmdg_t* h, const double* sigma_s, const double* sigma_a, const double* eps,
                       const double* q, const double* alpha, void* stream) {
  if (!h) return LMDG_INVALID_ARG;
  if (!sigma_s || !sigma_a || !eps || !q) return set_error(h, LMDG_INVALID_ARG, "NULL material array");
  if (alpha && h->dim == 3) return set_error(h, LMDG_UNSUPPORTED, "inflow data on 3D meshes");
  hipStream_t st = (hipStream_t)stream;
  const long long nc = h->ncell;
  std::vector<double> ss(nc), sa(nc), ep(nc), qq(nc);
  int rc = LMDG_OK;
  const double* src[4] = {sigma_s, sigma_a, eps, q};
  std::vector<double>* dst[4] = {&ss, &sa, &ep, &qq};
  for (int k = 0; k < 4 && rc == LMDG_OK; ++k)
    rc = check_hip(h, hipMemcpyAsync(dst[k]->data(), src[k], nc * sizeof(double), hipMemcpyDeviceToHost, st),
                   "read materials");
  if (rc == LMDG_OK) rc = check_hip(h, hipStreamSynchronize(st), "read materials");
  if (rc != LMDG_OK) return rc;
  std::vector<double> sigtA(nc), scatA(nc), absA(nc), qA(nc), epsA(nc);
  for (long long p = 0; p < nc; ++p) {
    if (!std::isfinite(ss[p]) || !std::isfinite(sa[p]) || !std::isfinite(ep[p]) || !std::isfinite(qq[p]))
      return set_error(h, LMDG_NONFINITE, "non-finite material value at cell " + std::to_string(p));
    if (ss[p] < 0 || sa[p] < 0 || !(ep[p] > 0))
      return set_error(h, LMDG_INVALID_ARG, "sigma < 0 or eps <= 0 at cell " + std::to_string(p));
    // eq-main: sigma_t = sigma_s/eps + eps sigma_a, scattering sigma_s/eps, source eps q
    sigtA[p] = (ss[p] / ep[p] + ep[p] * sa[p]) * h->area;
    scatA[p] = ss[p] / ep[p] * h->area;
    absA[p] = ep[p] * sa[p] * h->area;
    qA[p] = ep[p] * qq[p] * h->area;
    epsA[p] = ep[p] * h->area;
  }
  double** tgt[5] = {&h->d_sigtA, &h->d_scatA, &h->d_absA, &h->d_qA, &h->d_epsA};
  std::vector<double>* vals[5] = {&sigtA, &scatA, &absA, &qA, &epsA};
  for (int k = 0; k < 5 && rc == LMDG_OK; ++k) {
    if (!*tgt[k]) rc = check_hip(h, hipMalloc((void**)tgt[k], nc * sizeof(double)), "hipMalloc materials");
    if (rc == LMDG_OK)
      rc = check_hip(h, hipMemcpyAsync(*tgt[k], vals[k]->data(), nc * sizeof(double), hipMemcpyHostToDevice, st),
                     "write materials");
  }
  if (rc == LMDG_OK) rc = check_hip(h, hipStreamSynchronize(st), "write materials");
  if (rc == LMDG_OK) {
    h->have_mat = true;
    h->mat_version += 1;
    h->n_rhs = 1;
    h->h_eps = ep;
    clear_source_data(h, false);
    if (alpha) rc = set_alpha(h, alpha, st);
    if (rc != LMDG_OK) clear_source_data(h, false);
  }
  return rc;
}

int lmdg_set_source_moments(lmdg_t* h, int per_direction, const double* qm, void* stream) {
  if (!h) return LMDG_INVALID_ARG;
  if (!h->have_mat) return set_error(h, LMDG_INVALID_ARG, "materials not set");
  if (!qm || (per_direction != 0 && per_direction != 1)) return set_error(h, LMDG_INVALID_ARG, "bad source moments");
  if (h->dim != 2) return set_error(h, LMDG_UNSUPPORTED, "source moments on 3D meshes");
  hipStream_t st = (hipStream_t)stream;
  const long long nc = h->ncell;
  const int nd = per_direction ? h->ndir : 1;
  std::vector<double> m((size_t)nd * 4 * nc);
  int rc = check_hip(h, hipMemcpyAsync(m.data(), qm, m.size() * sizeof(double), hipMemcpyDeviceToHost, st),
                     "read source moments");
  if (rc == LMDG_OK) rc = check_hip(h, hipStreamSynchronize(st), "read source moments");
  if (rc != LMDG_OK) return rc;
  for (size_t e = 0; e < m.size(); ++e) {
    if (!std::isfinite(m[e])) return set_error(h, LMDG_NONFINITE, "non-finite source moment");
    m[e] *= h->h_eps[e % nc] * h->area;  // eps int_K q b_r = eps |K| q_r
  }
  rc = ensure_rhs_capacity(h, 1);
  if (rc != LMDG_OK) return rc;
  clear_source_data(h, true);
  h->n_rhs = 1;
  std::vector<double> q0(nc, 0.0), sq1(3 * (size_t)nc, 0.0);
  if (!per_direction) {
    std::copy(m.begin(), m.begin() + nc, q0.begin());
    std::copy(m.begin() + nc, m.end(), sq1.begin());
    rc = upload(h, &h->d_qS, sq1, st);
  } else {
    // per-direction moments go to the sweep whole; the isotropic constant is zero
    for (int l = 0; l < h->ndir; ++l)
      for (size_t e = 0; e < 3 * (size_t)nc; ++e) sq1[e] += h->w[l] * m[((size_t)l * 4) * nc + nc + e];
    rc = upload(h, &h->d_qdir, m, st);
  }
  if (rc == LMDG_OK) rc = upload(h, &h->d_sq1, sq1, st);
  if (rc == LMDG_OK)
    rc = check_hip(h, hipMemcpyAsync(h->d_qA, q0.data(), nc * sizeof(double), hipMemcpyHostToDevice, st),
                   "write source");
  if (rc == LMDG_OK) rc = check_hip(h, hipStreamSynchronize(st), "write source");
  if (rc != LMDG_OK) clear_source_data(h, true);
  return rc;
}

int lmdg_set_sources(lmdg_t* h, int n_rhs, const double* q, void* stream) {
  if (!h) return LMDG_INVALID_ARG;
  if (!h->have_mat) return set_error(h, LMDG_INVALID_ARG, "materials not set");
  if (!q || n_rhs < 1 || n_rhs > lmdg::kMaxRhs) return set_error(h, LMDG_INVALID_ARG, "bad source arguments");
  hipStream_t st = (hipStream_t)stream;
  const long long nc = h->ncell;
  std::vector<double> qq((size_t)n_rhs * nc);
  int rc = check_hip(h, hipMemcpyAsync(qq.data(), q, qq.size() * sizeof(double), hipMemcpyDeviceToHost, st),
                     "read sources");
  if (rc == LMDG_OK) rc = check_hip(h, hipStreamSynchronize(st), "read sources");
  if (rc != LMDG_OK) return rc;
  for (size_t e = 0; e < qq.size(); ++e) {
    if (!std::isfinite(qq[e])) return set_error(h, LMDG_NONFINITE, "non-finite source value");
    qq[e] = h->h_eps[e % nc] * qq[e] * h->area;  // eps q |K|, as lmdg_set_materials forms it
  }
  rc = ensure_rhs_capacity(h, n_rhs);
  if (rc != LMDG_OK) return rc;
  clear_source_data(h, true);
  rc = check_hip(h, hipMemcpyAsync(h->d_qA, qq.data(), qq.size() * sizeof(double), hipMemcpyHostToDevice, st),
                 "write sources");
  if (rc == LMDG_OK) rc = check_hip(h, hipStreamSynchronize(st), "write sources");
  if (rc == LMDG_OK) h->n_rhs = n_rhs;
  return rc;
}

}  // extern "C"

namespace {

int check_call(lmdg_t* h, int scheme, int prec) {
  if (!h) return LMDG_INVALID_ARG;
  if (scheme < LMDG_SCHEME_STD || scheme > LMDG_SCHEME_RLMDG)
    return set_error(h, LMDG_INVALID_ARG, "unknown scheme");
  if (prec != LMDG_PREC_FP64 && prec != LMDG_PREC_FP32) return set_error(h, LMDG_INVALID_ARG, "unknown precision");
  if (!h->have_mat) return set_error(h, LMDG_INVALID_ARG, "materials not set");
  return LMDG_OK;
}

// K x in the defect form (see lm_source / std_source): the same operator as
// eq-nonrec-block / eq-sndg-phi, arranged so that no O(sigma_s/eps) terms cancel
// after the sweep; this is what keeps FP32 sweeps usable at small eps.
int apply_op(lmdg_t* h, int scheme, int prec, const double* x, double* y, hipStream_t st) {
  if (h->adj_rlm) {
    // adjoint of RLMDG: K' X' = [X_0 - P_0 mu ; B_11 X'_1 - Sigma L_10 mu], mu the adjoint
    // sweep of the source formed from X' (adj_rlm_source_kernel)
    lmdg::launch_adj_rlm_source(h, x, nullptr, st);
    int rc = lmdg::launch_sweep(h, LMDG_SCHEME_RLMDG, prec, nullptr, false, nullptr, st, false);
    if (rc != LMDG_OK) return rc;
    lmdg::launch_combine(h, LMDG_SCHEME_RLMDG, prec, lmdg::kApply, x, y, st);
    return check_hip(h, hipGetLastError(), "combine");
  }
  // the reconstruction variants of RLMDG use the plain form (eq-nonrec-block applied as
  // printed: K x = [x_0 - P_0 psi ; B_11 x_1 - G psi])
  // the 3D standard scheme has the plain form only
  const bool defect = !(scheme == LMDG_SCHEME_RLMDG && h->recon_flags != 0) && !(h->dim == 3 && scheme == LMDG_SCHEME_STD);
  int rc = lmdg::launch_sweep(h, scheme, prec, x, false, nullptr, st, defect, 0xF, false, false);
  if (rc != LMDG_OK) return rc;
  lmdg::launch_combine(h, scheme, prec, defect ? lmdg::kApplyDefect : lmdg::kApply, x, y, st);
  return check_hip(h, hipGetLastError(), "combine");
}

int read_error_flag(lmdg_t* h, hipStream_t st) {
  int flag = 0;
  int rc = check_hip(h, hipMemcpyAsync(&flag, h->ws.err, sizeof(int), hipMemcpyDeviceToHost, st), "read flag");
  if (rc == LMDG_OK) rc = check_hip(h, hipStreamSynchronize(st), "read flag");
  if (rc == LMDG_OK && flag) {
    hipMemsetAsync(h->ws.err, 0, sizeof(int), st);
    return set_error(h, LMDG_HIP_ERROR, "sweep wait exceeded its spin limit");
  }
  return rc;
}

int ensure_small(lmdg_t* h, size_t doubles) {
  if (h->small_doubles >= doubles) return LMDG_OK;
  if (h->d_small) hipFree(h->d_small);
  if (h->h_small) hipHostFree(h->h_small);
  h->d_small = nullptr;
  h->h_small = nullptr;
  h->small_doubles = 0;
  int rc = check_hip(h, hipMalloc((void**)&h->d_small, doubles * sizeof(double)), "hipMalloc small");
  if (rc == LMDG_OK) rc = check_hip(h, hipHostMalloc((void**)&h->h_small, doubles * sizeof(double)), "pinned");
  if (rc == LMDG_OK) h->small_doubles = doubles;
  return rc;
}

// Workspace of one GMRES call, in doubles: the basis (mt + 1 vectors of NT values, FP64,
// or FP32 with an FP32 operator), r; with augmentation k stored corrections, their
// images, the cycle's correction and its image; with the preconditioner two more; with
// an FP32 basis the new Krylov vector and the operator's input in FP64.
size_t krylov_basis_doubles(int mt, bool lowv, long long NT) {
  return lowv ? ((size_t)(mt + 1) * NT + 1) / 2 : (size_t)(mt + 1) * NT;
}
size_t krylov_doubles(int mt, int ka, bool pc, bool lowv, long long NT) {
  return krylov_basis_doubles(mt, lowv, NT) +
         (size_t)(1 + (ka > 0 ? 2 * ka + 2 : 0) + (pc ? 2 : 0) + (lowv ? 2 : 0)) * NT;
}

int ensure_krylov(lmdg_t* h, size_t doubles) {
  if (h->krylov_doubles >= doubles) return LMDG_OK;
  if (h->d_krylov) hipFree(h->d_krylov);
  h->d_krylov = nullptr;
  h->krylov_doubles = 0;
  int rc = check_hip(h, hipMalloc((void**)&h->d_krylov, doubles * sizeof(double)), "hipMalloc krylov");
  if (rc == LMDG_OK) h->krylov_doubles = doubles;
  return rc;
}

// Scratch layout of d_small / h_small for nr right-hand sides (offsets in doubles):
//   coef   2 (kMaxRestart + 2) nr   GMRES coefficients (device) / both CGS passes (host)
//   part   kDotBlocks (kMaxRestart + 2) nr   partial sums of the dot kernels (device)
//   scal   nr                       per-segment scale factors
//   res    nr                       dot / norm results
constexpr int kMaxRestart = 250;
struct SmallLayout {
  size_t coef, part, scal, res, total;
};
SmallLayout small_layout(int nr) {
  SmallLayout L;
  L.coef = 0;
  L.part = (size_t)2 * (kMaxRestart + 2) * nr;
  L.scal = L.part + (size_t)lmdg::dots_partials() * (kMaxRestart + 2) * nr;
  L.res = L.scal + nr;
  L.total = L.res + nr + 8;
  return L;
}

// Per-segment dot products a[rz] . b[rz] (nr segments of length n) into out[0..nr),
// synchronising the stream.
int seg_dots(lmdg_t* h, const double* a, const double* b, long long n, int nr, double* out, hipStream_t st) {
  const SmallLayout L = small_layout(nr);
  int rc = ensure_small(h, L.total);
  if (rc != LMDG_OK) return rc;
  lmdg::vec_dots(a, n * nr, 1, b, n, h->d_small + L.part, h->d_small + L.res, st, nr);
  rc = check_hip(h, hipMemcpyAsync(h->h_small + L.res, h->d_small + L.res, nr * sizeof(double),
                                   hipMemcpyDeviceToHost, st), "dots");
  if (rc == LMDG_OK) rc = check_hip(h, hipStreamSynchronize(st), "dots");
  if (rc == LMDG_OK) std::copy(h->h_small + L.res, h->h_small + L.res + nr, out);
  return rc;
}

// ||v[rz]||_2 for every segment.
int seg_norms(lmdg_t* h, const double* v, long long n, int nr, double* out, hipStream_t st) {
  int rc = seg_dots(h, v, v, n, nr, out, st);
  for (int k = 0; k < nr; ++k) out[k] = std::sqrt(std::max(0.0, out[k]));
  return rc;
}

int dot(lmdg_t* h, const double* a, const double* b, long long n, double* out, hipStream_t st) {
  return seg_dots(h, a, b, n, 1, out, st);
}

// LMDG_VERBOSE=1 in the environment prints solver progress to stderr.
bool verbose() {
  static const bool v = [] {
    const char* e = std::getenv("LMDG_VERBOSE");
    return e && e[0] && e[0] != '0';
  }();
  return v;
}

struct GmresStats {
  int iterations = 0, restarts = 0;
  double apply_ms = 0;
  // LGMRES store (pairs z, K z in the Krylov workspace): filled pairs and the next ring
  // slot.  It persists across the gmres calls that share one GmresStats, so the inner
  // solves of iterative refinement (same FP32 operator) keep the earlier passes' pairs.
  int n_aug = 0, aug_next = 0;
  int reorth = 0;  // Arnoldi steps that took a second Gram-Schmidt pass
};

// Restarted GMRES(m) with classical Gram-Schmidt (a second pass where the first
// cancelled), FP64 vectors, for the handle's nr right-hand sides at once: nr
// independent GMRES instances (own Hessenberg
// matrices, rotations and stopping tests) share every operator application.  Solves
// K_prec x = b from x (in/out); stops when every true FP64-operator residual
// ||b - K x|| <= rtol ||b|| (true_prec) or after max_iter applications.  relres is
// the largest relative residual over the right-hand sides.
//
// With h->augment = k > 0 each cycle also searches the directions of the last k
// cycles' corrections (LGMRES, Baker, Jessup and Manteuffel 2005): after the m Krylov
// steps the Arnoldi process continues with the stored images K z of those corrections
// (no operator application), the search directions being the Krylov vectors and the
// z's (flexible GMRES form, K Z = V H).  The new correction z = Z y and its image
// K z = V H y enter the store, so restarts keep what the earlier cycles learned.  The
// store lives in stats and carries over to the next call with the same stats and
// operator precision.
int gmres(lmdg_t* h, int scheme, int prec, int true_prec, const double* b, double* x, double rtol, int m,
          int max_iter, hipStream_t st, GmresStats& stats, double& relres, bool& converged) {
  const int nr = h->n_rhs;
  const long long N = (long long)h->np * h->ncell;  // one right-hand side
  const long long NT = N * nr;
  const int ka_max = std::max(0, std::min(h->augment, kMaxRestart - m));
  const int mt = m + ka_max;                          // steps per cycle at most
  const SmallLayout L = small_layout(nr);
  // right preconditioning (lmdg_set_preconditioner) where it covers the system
  const bool pc = h->pc_kind != LMDG_PRECOND_NONE && lmdg::pc_supported(h, scheme, nullptr);
  // with an FP32 operator (the inner solves of mode MIXED) the basis is stored in FP32:
  // the orthogonalisation reads it twice per step, and the inner solves aim at a few
  // digits only; products, sums, the new vector and the corrections stay FP64
  const bool lowv = prec == LMDG_PREC_FP32;
  const size_t basis_d = krylov_basis_doubles(mt, lowv, NT);
  const double* prev_krylov = h->d_krylov;
  int rc = ensure_krylov(h, krylov_doubles(mt, ka_max, pc, lowv, NT));
  if (h->d_krylov != prev_krylov) stats.n_aug = stats.aug_next = 0;  // store lost with the old buffer
  if (rc == LMDG_OK) rc = ensure_small(h, L.total);
  if (rc != LMDG_OK) return rc;
  double* V = lowv ? nullptr : h->d_krylov;                   // mt + 1 basis vectors of length NT
  float* Vf = lowv ? reinterpret_cast<float*>(h->d_krylov) : nullptr;
  double* r = h->d_krylov + basis_d;       // residual work vector
  double* Z = r + NT;                      // ka_max stored corrections
  double* AZ = Z + (size_t)ka_max * NT;    // their images
  double* dz = ka_max > 0 ? AZ + (size_t)ka_max * NT : x;  // this cycle's correction (x itself
  double* adz = dz + NT;                                     // without augmentation), its image
  double* tail = r + (size_t)(1 + (ka_max > 0 ? 2 * ka_max + 2 : 0)) * NT;
  double* pt = tail;                                         // preconditioner input / output
  double* pz = pt + NT;
  double* wv = tail + (pc ? 2 : 0) * NT;   // FP32 basis: the new Krylov vector in FP64
  double* vin = wv + NT;                   // FP32 basis: the basis vector the operator takes
  // basis operations for either storage
  auto basis_dots = [&](int nv, const double* w) {
    if (lowv) lmdg::vec_dots(Vf, NT, nv, w, N, h->d_small + L.part, h->d_small + L.coef, st, nr);
    else lmdg::vec_dots(V, NT, nv, w, N, h->d_small + L.part, h->d_small + L.coef, st, nr);
  };
  auto basis_axpy = [&](double* w, int nv, const double* coef, double sign) {
    if (lowv) lmdg::vec_axpy_multi(w, Vf, NT, nv, coef, sign, N, st, nr);
    else lmdg::vec_axpy_multi(w, V, NT, nv, coef, sign, N, st, nr);
  };
  auto basis_store = [&](int j, const double* src, const double* scale) {  // V_j = scale * src
    if (lowv) lmdg::vec_scale_seg(Vf + (size_t)j * NT, src, scale, N, nr, st);
    else lmdg::vec_scale_seg(V + (size_t)j * NT, src, scale, N, nr, st);
  };
  auto basis_vec = [&](int j) -> const double* {  // V_j in FP64 (widened into vin)
    if (!lowv) return V + (size_t)j * NT;
    lmdg::vec_widen(vin, Vf + (size_t)j * NT, NT, st);
    return vin;
  };
  double* dcoef = h->d_small + L.coef;
  double* dscal = h->d_small + L.scal;
  double* part = h->d_small + L.part;
  double* hc = h->h_small + L.coef;        // first pass at 0, second at (mt + 1) nr
  double* hscal = h->h_small + L.scal;
  std::vector<double> bnorm(nr), beta(nr), hn(nr), zn(nr);
  rc = seg_norms(h, b, N, nr, bnorm.data(), st);
  if (rc != LMDG_OK) return rc;
  converged = false;
  relres = 1.0;
  const size_t hsz = (size_t)(mt + 1) * mt;
  std::vector<std::vector<double>> H(nr, std::vector<double>(hsz)), H0(nr, std::vector<double>(hsz)),
      cs(nr, std::vector<double>(mt)), sn(nr, std::vector<double>(mt)), g(nr, std::vector<double>(mt + 1));
  std::vector<int> kr(nr);
  std::vector<char> done(nr);
  std::vector<double> y(mt);
  std::vector<std::vector<double>> ys(nr, std::vector<double>(mt, 0.0));
  int& n_aug = stats.n_aug;                // stored corrections, ring position
  int& aug_next = stats.aug_next;
  if (n_aug > ka_max || aug_next >= std::max(ka_max, 1)) n_aug = aug_next = 0;
  double prev_relres = -1.0;
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  auto timed_apply = [&](int p, const double* in, double* out) {
    hipEventRecord(e0, st);
    int r2 = apply_op(h, scheme, p, in, out, st);
    hipEventRecord(e1, st);
    return r2;
  };
  auto add_time = [&]() {
    float ms = 0;
    hipEventSynchronize(e1);
    hipEventElapsedTime(&ms, e0, e1);
    stats.apply_ms += ms;
  };
  auto upload_scales = [&]() {
    return check_hip(h, hipMemcpyAsync(dscal, hscal, nr * sizeof(double), hipMemcpyHostToDevice, st), "scales");
  };
  while (rc == LMDG_OK) {
    // true residuals with the FP64 (or requested) operator
    rc = timed_apply(true_prec, x, r);
    if (rc != LMDG_OK) break;
    lmdg::vec_axpby(r, 1.0, b, -1.0, NT, st);  // r = b - K x
    rc = seg_norms(h, r, N, nr, beta.data(), st);
    add_time();
    if (rc != LMDG_OK) break;
    relres = 0.0;
    bool finite = true;
    for (int k = 0; k < nr; ++k) {
      finite = finite && std::isfinite(beta[k]);
      relres = std::max(relres, bnorm[k] > 0 ? beta[k] / bnorm[k] : 0.0);
    }
    if (verbose())
      std::fprintf(stderr, "lmdg GMRES(%d+%d) %s: restart %d, %d its, true rel residual %.3e (max over %d rhs)\n", m,
                   n_aug, prec == LMDG_PREC_FP64 ? "fp64" : "fp32", stats.restarts, stats.iterations, relres, nr);
    if (!finite) { rc = set_error(h, LMDG_NONFINITE, "non-finite residual"); break; }
    if (relres <= rtol) { converged = true; break; }
    if (stats.iterations >= max_iter) break;
    // an FP32 inner solve of the refinement loop returns once a restart cycle no
    // longer reduces its own true residual (the FP32 operator's accuracy floor)
    if (prec == LMDG_PREC_FP32 && prev_relres > 0 && relres >= prev_relres) break;
    prev_relres = relres;
    stats.restarts += 1;
    for (int k = 0; k < nr; ++k) {
      std::fill(g[k].begin(), g[k].end(), 0.0);
      g[k][0] = beta[k];
      kr[k] = 0;
      done[k] = beta[k] == 0.0 || beta[k] <= 0.5 * rtol * bnorm[k];
      hscal[k] = done[k] ? 0.0 : 1.0 / beta[k];
    }
    rc = upload_scales();
    if (rc != LMDG_OK) break;
    basis_store(0, r, dscal);
    const int steps = m + n_aug;
    for (int j = 0; j < steps; ++j) {
      const bool krylov = j < m;
      if (krylov && stats.iterations >= max_iter) break;
      double* w = lowv ? wv : V + (size_t)(j + 1) * NT;
      if (krylov) {
        const double* vj = basis_vec(j);
        if (pc) {  // w = K M^{-1} v_j
          rc = lmdg::pc_apply(h, scheme, vj, pz, st);
          if (rc != LMDG_OK) break;
        }
        rc = timed_apply(prec, pc ? pz : vj, w);
        if (rc != LMDG_OK) break;
        stats.iterations += 1;
      } else {
        // image of a stored correction, newest first
        const int slot = ((aug_next - 1 - (j - m)) % ka_max + ka_max) % ka_max;
        lmdg::vec_copy(w, AZ + (size_t)slot * NT, NT, st);
      }
      // classical Gram-Schmidt, coefficients kept on the device; a second pass only where
      // the first cancelled: ||w'|| < ||w|| / sqrt(2), i.e. ||w'||^2 < sum_i h_i^2 with
      // w' = w - V h (Daniel, Gragg, Kaufman and Stewart 1976)
      basis_dots(j + 1, w);
      basis_axpy(w, j + 1, dcoef, -1.0);
      rc = check_hip(h, hipMemcpyAsync(hc, dcoef, (j + 1) * nr * sizeof(double), hipMemcpyDeviceToHost, st), "h");
      if (rc != LMDG_OK) break;
      rc = seg_norms(h, w, N, nr, hn.data(), st);  // synchronises: hc is valid afterwards
      if (rc != LMDG_OK) break;
      bool second = false;
      for (int k = 0; k < nr && !second; ++k) {
        if (done[k]) continue;
        double hh = 0.0;
        for (int i = 0; i <= j; ++i) hh += hc[(size_t)i * nr + k] * hc[(size_t)i * nr + k];
        second = !(hn[k] * hn[k] >= hh);
      }
      double* hc2 = hc + (size_t)(mt + 1) * nr;
      if (second) {
        basis_dots(j + 1, w);
        basis_axpy(w, j + 1, dcoef, -1.0);
        rc = check_hip(h, hipMemcpyAsync(hc2, dcoef, (j + 1) * nr * sizeof(double), hipMemcpyDeviceToHost, st),
                       "h2");
        if (rc != LMDG_OK) break;
        rc = seg_norms(h, w, N, nr, hn.data(), st);
        if (rc != LMDG_OK) break;
        stats.reorth += 1;
      } else {
        std::fill(hc2, hc2 + (size_t)(j + 1) * nr, 0.0);
      }
      if (krylov) add_time();
      bool all_done = true;
      for (int k = 0; k < nr; ++k) {
        if (done[k]) {  // finished at an earlier step: its segments stay zero
          hscal[k] = 0.0;
          continue;
        }
        if (!std::isfinite(hn[k])) { rc = set_error(h, LMDG_NONFINITE, "non-finite Krylov vector"); break; }
        std::vector<double>& Hk = H[k];
        for (int i = 0; i <= j; ++i)
          Hk[(size_t)i * mt + j] = hc[(size_t)i * nr + k] + hc[(size_t)(mt + 1) * nr + (size_t)i * nr + k];
        Hk[(size_t)(j + 1) * mt + j] = hn[k];
        for (int i = 0; i <= j + 1; ++i) H0[k][(size_t)i * mt + j] = Hk[(size_t)i * mt + j];
        for (int i = 0; i < j; ++i) {  // previous rotations
          const double a = Hk[(size_t)i * mt + j], c = Hk[(size_t)(i + 1) * mt + j];
          Hk[(size_t)i * mt + j] = cs[k][i] * a + sn[k][i] * c;
          Hk[(size_t)(i + 1) * mt + j] = -sn[k][i] * a + cs[k][i] * c;
        }
        const double a = Hk[(size_t)j * mt + j], c = Hk[(size_t)(j + 1) * mt + j];
        const double rr = std::hypot(a, c);
        hscal[k] = hn[k] > 0.0 ? 1.0 / hn[k] : 0.0;
        if (rr == 0.0) {
          // direction already in the span (only a stored correction can be): drop
          // the column and stop this right-hand side's cycle
          done[k] = 1;
          continue;
        }
        cs[k][j] = a / rr;
        sn[k][j] = c / rr;
        Hk[(size_t)j * mt + j] = rr;
        Hk[(size_t)(j + 1) * mt + j] = 0.0;
        g[k][j + 1] = -sn[k][j] * g[k][j];
        g[k][j] = cs[k][j] * g[k][j];
        kr[k] = j + 1;
        if (std::fabs(g[k][j + 1]) <= 0.5 * rtol * bnorm[k] || hn[k] == 0.0) done[k] = 1;
        all_done = all_done && done[k];
      }
      if (rc != LMDG_OK) break;
      // normalise the new basis vector of every right-hand side active at this step
      // (the image of the cycle's correction uses it also when that one just finished)
      rc = upload_scales();
      if (rc != LMDG_OK) break;
      basis_store(j + 1, w, dscal);
      if (all_done) break;
    }
    if (rc != LMDG_OK) break;
    // per right-hand side: H_k y_k = g_k (upper triangular, k_r columns)
    int kmax = 0;
    for (int k = 0; k < nr; ++k) kmax = std::max(kmax, kr[k]);
    if (kmax == 0) continue;
    for (int k = 0; k < nr; ++k) {
      std::fill(ys[k].begin(), ys[k].end(), 0.0);
      const int kk = kr[k];
      const std::vector<double>& Hk = H[k];
      for (int i = kk - 1; i >= 0; --i) {
        double acc = g[k][i];
        for (int jj = i + 1; jj < kk; ++jj) acc -= Hk[(size_t)i * mt + jj] * y[jj];
        y[i] = acc / Hk[(size_t)i * mt + i];
      }
      for (int i = 0; i < kk; ++i) ys[k][i] = y[i];
    }
    // correction dz = Z y: Krylov part sum_{j<m} y_j V_j, augmented part sum_l y_{m+l} z_l
    const int nkry = std::min(kmax, m);
    std::fill(hc, hc + (size_t)(mt + 1) * nr, 0.0);
    for (int k = 0; k < nr; ++k)
      for (int i = 0; i < nkry; ++i) hc[(size_t)i * nr + k] = ys[k][i];
    rc = check_hip(h, hipMemcpyAsync(dcoef, hc, (size_t)nkry * nr * sizeof(double), hipMemcpyHostToDevice, st), "y");
    if (rc != LMDG_OK) break;
    if (pc) {
      // Krylov part of the correction: M^{-1} (sum_j y_j V_j)
      lmdg::vec_fill(pt, 0.0, NT, st);
      basis_axpy(pt, nkry, dcoef, 1.0);
      rc = lmdg::pc_apply(h, scheme, pt, pz, st);
      if (rc != LMDG_OK) break;
      if (ka_max > 0) lmdg::vec_copy(dz, pz, NT, st);
      else lmdg::vec_axpby(x, 1.0, pz, 1.0, NT, st);
    } else {
      if (ka_max > 0) lmdg::vec_fill(dz, 0.0, NT, st);
      basis_axpy(dz, nkry, dcoef, 1.0);
    }
    if (kmax > m) {
      // stored corrections: coefficients by ring slot (step m + l used slot aug_next - 1 - l)
      double* hz = hc + (size_t)(mt + 1) * nr;
      std::fill(hz, hz + (size_t)ka_max * nr, 0.0);
      for (int l = 0; l + m < kmax; ++l) {
        const int slot = ((aug_next - 1 - l) % ka_max + ka_max) % ka_max;
        for (int k = 0; k < nr; ++k) hz[(size_t)slot * nr + k] = ys[k][m + l];
      }
      double* dz_coef = dcoef + (size_t)(mt + 1) * nr;
      rc = check_hip(h, hipMemcpyAsync(dz_coef, hz, (size_t)ka_max * nr * sizeof(double), hipMemcpyHostToDevice,
                                       st), "y aug");
      if (rc != LMDG_OK) break;
      lmdg::vec_axpy_multi(dz, Z, NT, n_aug, dz_coef, 1.0, N, st, nr);
    }
    if (ka_max > 0) lmdg::vec_axpby(x, 1.0, dz, 1.0, NT, st);
    rc = check_hip(h, hipStreamSynchronize(st), "update");  // the host coefficients are reused
    if (rc != LMDG_OK || ka_max == 0) continue;
    // image K dz = V (H0 y) from the unrotated Hessenberg columns, then store the
    // normalised pair (z, K z) in the ring
    std::fill(hc, hc + (size_t)(mt + 1) * nr, 0.0);
    for (int k = 0; k < nr; ++k) {
      const int kk = kr[k];
      for (int i = 0; i <= kk; ++i) {
        double acc = 0.0;
        for (int jj = 0; jj < kk; ++jj) acc += (i <= jj + 1 ? H0[k][(size_t)i * mt + jj] : 0.0) * ys[k][jj];
        hc[(size_t)i * nr + k] = acc;
      }
    }
    rc = check_hip(h, hipMemcpyAsync(dcoef, hc, (size_t)(kmax + 1) * nr * sizeof(double), hipMemcpyHostToDevice,
                                     st), "hy");
    if (rc != LMDG_OK) break;
    lmdg::vec_fill(adz, 0.0, NT, st);
    basis_axpy(adz, kmax + 1, dcoef, 1.0);
    rc = seg_norms(h, dz, N, nr, zn.data(), st);
    if (rc != LMDG_OK) break;
    for (int k = 0; k < nr; ++k) hscal[k] = zn[k] > 0 ? 1.0 / zn[k] : 0.0;
    rc = upload_scales();
    if (rc != LMDG_OK) break;
    lmdg::vec_scale_seg(Z + (size_t)aug_next * NT, dz, dscal, N, nr, st);
    lmdg::vec_scale_seg(AZ + (size_t)aug_next * NT, adz, dscal, N, nr, st);
    aug_next = (aug_next + 1) % ka_max;
    n_aug = std::min(n_aug + 1, ka_max);
    rc = check_hip(h, hipStreamSynchronize(st), "augment");
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc == LMDG_OK) rc = read_error_flag(h, st);
  return rc;
}

}  // namespace

namespace lmdg {
// K x for entry points outside this file (lmdg_apply_noalloc).
int apply_op_impl(lmdg_handle* h, int scheme, int prec, const double* x, double* y, hipStream_t st) {
  return apply_op(h, scheme, prec, x, y, st);
}
}  // namespace lmdg

extern "C" {

int lmdg_sweep(lmdg_t* h, int scheme, int prec, const double* x, int use_q, double* out, double* psi,
               void* stream) {
  int rc = check_call(h, scheme, prec);
  if (rc != LMDG_OK) return rc;
  if (!out) return set_error(h, LMDG_INVALID_ARG, "NULL output");
  hipStream_t st = (hipStream_t)stream;
  rc = lmdg::launch_sweep(h, scheme, prec, x, use_q != 0, psi, st);
  if (rc != LMDG_OK) return rc;
  lmdg::launch_sum_quadrants(h, scheme, prec, out, st);
  return check_hip(h, hipGetLastError(), "sweep");
}

int lmdg_apply(lmdg_t* h, int scheme, int prec, const double* x, double* y, void* stream) {
  int rc = check_call(h, scheme, prec);
  if (rc != LMDG_OK) return rc;
  if (!x || !y) return set_error(h, LMDG_INVALID_ARG, "NULL vector");
  return apply_op(h, scheme, prec, x, y, (hipStream_t)stream);
}

int lmdg_rhs(lmdg_t* h, int scheme, int prec, double* b, void* stream) {
  int rc = check_call(h, scheme, prec);
  if (rc != LMDG_OK) return rc;
  if (!b) return set_error(h, LMDG_INVALID_ARG, "NULL vector");
  hipStream_t st = (hipStream_t)stream;
  if (h->adj_rlm) {  // adjoint of RLMDG (inside lmdg_adjoint_solve): source from the detector
    lmdg::launch_adj_rlm_source(h, nullptr, h->adj_det, st);
    rc = lmdg::launch_sweep(h, LMDG_SCHEME_RLMDG, prec, nullptr, false, nullptr, st);
    if (rc != LMDG_OK) return rc;
    lmdg::launch_combine(h, LMDG_SCHEME_RLMDG, prec, lmdg::kRhs, nullptr, b, st);
    return check_hip(h, hipGetLastError(), "rhs");
  }
  rc = lmdg::launch_sweep(h, scheme, prec, nullptr, true, nullptr, st, false, 0xF, false, false);
  if (rc != LMDG_OK) return rc;
  lmdg::launch_combine(h, scheme, prec, lmdg::kRhs, nullptr, b, st);
  return check_hip(h, hipGetLastError(), "rhs");
}

int lmdg_recover(lmdg_t* h, int scheme, int prec, const double* x, double* phi, double* psi, void* stream) {
  int rc = check_call(h, scheme, prec);
  if (rc != LMDG_OK) return rc;
  if (!x || !phi) return set_error(h, LMDG_INVALID_ARG, "NULL vector");
  hipStream_t st = (hipStream_t)stream;
  if (h->adj_rlm) {  // adjoint of RLMDG: mu = sweep of the full source; [P_0 mu ; -X'_1]
    lmdg::launch_adj_rlm_source(h, x, h->adj_det, st);
    rc = lmdg::launch_sweep(h, LMDG_SCHEME_RLMDG, prec, nullptr, false, psi, st);
    if (rc != LMDG_OK) return rc;
    lmdg::launch_combine(h, LMDG_SCHEME_RLMDG, prec, lmdg::kRecover, x, phi, st);
    return check_hip(h, hipGetLastError(), "recover");
  }
  rc = lmdg::launch_sweep(h, scheme, prec, x, true, psi, st);
  if (rc != LMDG_OK) return rc;
  lmdg::launch_combine(h, scheme, prec, lmdg::kRecover, x, phi, st);
  return check_hip(h, hipGetLastError(), "recover");
}

// The solve behind lmdg_solve and lmdg_adjoint_solve.  rhs_x (nullable) is the
// moment vector the right-hand-side sweep takes (Step 1's -Sigma^T c term when the
// source has slope moments); cshift (nullable) is c, removed from x before recovery
// (Psi_0 = L_00^{-1}(M_0 X_0 + L_01 Sigma^T (X_1 - c) + Q_0), Phi_1 = c - X_1).
static int solve_impl(lmdg_t* h, int scheme, int mode, double tol, int restart, int max_iter, const double* x0,
                      double* x_out, double* phi_out, double* psi_out, lmdg_info* info, hipStream_t st,
                      const double* rhs_x, const double* cshift) {
  const int nr = h->n_rhs;
  int rc = ensure_small(h, small_layout(nr).total);
  if (rc != LMDG_OK) return rc;
  const auto t_start = std::chrono::steady_clock::now();
  const long long N = (long long)h->np * h->ncell * nr;  // all right-hand sides
  const long long N1 = (long long)h->np * h->ncell;
  double* b = h->ws.vec;
  double* r = h->ws.vec + N;
  double* d = h->ws.vec + 2 * N;
  if (!rhs_x) {
    rc = lmdg_rhs(h, scheme, LMDG_PREC_FP64, b, st);
  } else {
    rc = lmdg::launch_sweep(h, scheme, LMDG_PREC_FP64, rhs_x, true, nullptr, st, false, 0xF, false, false);
    if (rc == LMDG_OK) lmdg::launch_combine(h, scheme, LMDG_PREC_FP64, lmdg::kRhs, nullptr, b, st);
  }
  if (rc != LMDG_OK) return rc;
  if (x0) lmdg::vec_copy(x_out, x0, N, st); else lmdg::vec_fill(x_out, 0.0, N, st);
  GmresStats stats;
  double relres = 1.0;
  bool conv = false;
  int passes = 0;
  if (mode == LMDG_MODE_FP64) {
    passes = 1;
    rc = gmres(h, scheme, LMDG_PREC_FP64, LMDG_PREC_FP64, b, x_out, tol, restart, max_iter, st, stats, relres, conv);
  } else {
    // FP64 iterative refinement: r = b - K64 x; inner GMRES with FP32 sweeps on K d = r
    std::vector<double> bnorm(nr), rn(nr);
    rc = seg_norms(h, b, N1, nr, bnorm.data(), st);
    while (rc == LMDG_OK && stats.iterations < max_iter && passes < 100) {
      rc = apply_op(h, scheme, LMDG_PREC_FP64, x_out, r, st);
      if (rc != LMDG_OK) break;
      lmdg::vec_axpby(r, 1.0, b, -1.0, N, st);
      rc = seg_norms(h, r, N1, nr, rn.data(), st);
      if (rc != LMDG_OK) break;
      relres = 0.0;
      bool finite = true;
      for (int k = 0; k < nr; ++k) {
        finite = finite && std::isfinite(rn[k]);
        relres = std::max(relres, bnorm[k] > 0 ? rn[k] / bnorm[k] : 0.0);
      }
      if (!finite) { rc = set_error(h, LMDG_NONFINITE, "non-finite residual"); break; }
      if (relres <= tol) { conv = true; break; }
      passes += 1;
      lmdg::vec_fill(d, 0.0, N, st);
      // FP32 sweeps carry about 1e-6 relative error, so each pass asks for a few digits
      // (three unless lmdg_set_refinement says otherwise) and the FP64 residual of the
      // next pass corrects the rest
      const double inner = std::max(h->ir_inner, 0.5 * tol / relres);
      bool iconv = false;
      double irel = 1;
      const int before = stats.iterations;
      // max_iter bounds the cumulative count kept in stats
      rc = gmres(h, scheme, LMDG_PREC_FP32, LMDG_PREC_FP32, r, d, std::min(inner, 0.5), restart, max_iter, st,
                 stats, irel, iconv);
      if (verbose())
        std::fprintf(stderr, "lmdg IR pass %d: FP64 rel residual %.3e, inner %d its to %.3e (%s)\n", passes, relres,
                     stats.iterations - before, irel, iconv ? "converged" : "not converged");
      if (rc != LMDG_OK) break;
      lmdg::vec_axpby(x_out, 1.0, d, 1.0, N, st);
    }
  }
  if (rc == LMDG_OK && phi_out) {
    const double* xr = x_out;
    if (cshift) {
      double* t = h->ws.vec + 3 * N;
      lmdg::vec_copy(t, x_out, N, st);
      lmdg::vec_axpby(t, -1.0, cshift, 1.0, N, st);
      xr = t;
    }
    rc = lmdg_recover(h, scheme, LMDG_PREC_FP64, xr, phi_out, psi_out, st);
  }
  if (rc == LMDG_OK) rc = check_hip(h, hipStreamSynchronize(st), "solve");
  // the recovery sweep ran after the last flag check inside gmres
  if (rc == LMDG_OK) rc = read_error_flag(h, st);
  const double total =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  if (info) {
    info->iterations = stats.iterations;
    info->restarts = stats.restarts;
    info->ir_passes = passes;
    info->converged = conv ? 1 : 0;
    info->rel_residual = relres;
    info->time_total_ms = total;
    info->time_apply_ms = stats.apply_ms;
  }
  if (rc != LMDG_OK) return rc;
  return conv ? LMDG_OK : set_error(h, LMDG_NOT_CONVERGED, "tolerance not reached");
}

int lmdg_solve(lmdg_t* h, int scheme, int mode, double tol, int restart, int max_iter, const double* x0,
               double* x_out, double* phi_out, lmdg_info* info, void* stream) {
  int rc = check_call(h, scheme, LMDG_PREC_FP64);
  if (rc != LMDG_OK) return rc;
  if (!x_out || !(tol > 0) || restart < 1 || restart > 250 || max_iter < 1 ||
      (mode != LMDG_MODE_FP64 && mode != LMDG_MODE_MIXED))
    return set_error(h, LMDG_INVALID_ARG, "bad solve arguments");
  return solve_impl(h, scheme, mode, tol, restart, max_iter, x0, x_out, phi_out, nullptr, info, (hipStream_t)stream,
                    nullptr, nullptr);
}

// Conjugate gradients on B_11 c = f_1 (B_11 symmetric positive definite, Sec. 3.2);
// vectors in the moment-major layout with slot 0 held at zero.  Uses ws.vec[0..3).
static int cg_b11(lmdg_t* h, const double* f, double* c, double rtol, hipStream_t st) {
  const long long nc = h->ncell, N = (long long)h->np * nc;
  double* r = h->ws.vec;
  double* p = h->ws.vec + N;
  double* Ap = h->ws.vec + 2 * N;
  lmdg::vec_copy(r, f, N, st);
  lmdg::vec_fill(r, 0.0, nc, st);
  lmdg::vec_fill(c, 0.0, N, st);
  double rr;
  int rc = dot(h, r, r, N, &rr, st);
  if (rc != LMDG_OK) return rc;
  const double bn = std::sqrt(rr);
  if (bn == 0.0) return LMDG_OK;
  lmdg::vec_copy(p, r, N, st);
  for (int it = 0; it < 100000; ++it) {
    lmdg::launch_b11(h, p, Ap, st);
    double pAp;
    rc = dot(h, p, Ap, N, &pAp, st);
    if (rc != LMDG_OK) return rc;
    if (!(pAp > 0)) return set_error(h, LMDG_NONFINITE, "B_11 conjugate gradients broke down");
    const double alpha = rr / pAp;
    lmdg::vec_axpby(c, alpha, p, 1.0, N, st);
    lmdg::vec_axpby(r, -alpha, Ap, 1.0, N, st);
    double rr_new;
    rc = dot(h, r, r, N, &rr_new, st);
    if (rc != LMDG_OK) return rc;
    if (std::sqrt(rr_new) <= rtol * bn) return LMDG_OK;
    lmdg::vec_axpby(p, 1.0, r, rr_new / rr, N, st);
    rr = rr_new;
  }
  return set_error(h, LMDG_NOT_CONVERGED, "B_11 conjugate gradients did not converge");
}

int lmdg_adjoint_solve(lmdg_t* h, int scheme, int mode, const double* det, double tol, int restart, int max_iter,
                       double* g_sigma_s, double* g_sigma_a, double* g_q, double* J_out, lmdg_info* info,
                       void* stream) {
  int rc = check_call(h, scheme, LMDG_PREC_FP64);
  if (rc != LMDG_OK) return rc;
  const bool rlm = scheme == LMDG_SCHEME_RLMDG;
  if (rlm && h->recon_flags != 0)
    return set_error(h, LMDG_UNSUPPORTED, "the RLMDG adjoint covers the two-cell reconstruction only");
  if (h->dim != 2) return set_error(h, LMDG_UNSUPPORTED, "the adjoint solve is two-dimensional");
  if (h->slab) return set_error(h, LMDG_UNSUPPORTED, "adjoint of a slab handle");
  if (!det || !g_sigma_s || !g_sigma_a || !g_q || !J_out || !(tol > 0) || restart < 1 || restart > 250 ||
      max_iter < 1 || (mode != LMDG_MODE_FP64 && mode != LMDG_MODE_MIXED))
    return set_error(h, LMDG_INVALID_ARG, "bad adjoint arguments");
  for (int l = 0; l < h->ndir; ++l)
    if (h->neg_dir[l] < 0) return set_error(h, LMDG_INVALID_ARG, "quadrature is not centrally symmetric");
  if (h->n_rhs != 1) return set_error(h, LMDG_INVALID_ARG, "the adjoint solve takes one right-hand side");
  hipStream_t st = (hipStream_t)stream;
  const long long nc = h->ncell, N = (long long)h->np * nc;
  const int npsi = scheme == LMDG_SCHEME_STD ? 4 : 1;
  // angular fluxes of one quadrant at a time (forward and opposite-quadrant adjoint)
  const size_t psi_doubles = (size_t)h->dslots * npsi * nc;
  if (h->psi_doubles < psi_doubles) {
    if (h->d_psi_f) hipFree(h->d_psi_f);
    if (h->d_psi_a) hipFree(h->d_psi_a);
    h->d_psi_f = h->d_psi_a = nullptr;
    h->psi_doubles = 0;
    rc = check_hip(h, hipMalloc((void**)&h->d_psi_f, psi_doubles * sizeof(double)), "hipMalloc psi");
    if (rc == LMDG_OK) rc = check_hip(h, hipMalloc((void**)&h->d_psi_a, psi_doubles * sizeof(double)), "hipMalloc psi");
    if (rc != LMDG_OK) return rc;
    h->psi_doubles = psi_doubles;
  }
  if (!h->d_cvec) {
    rc = check_hip(h, hipMalloc((void**)&h->d_cvec, (size_t)6 * N * sizeof(double)), "hipMalloc adjoint vectors");
    if (rc != LMDG_OK) return rc;
  }
  if (rlm && !h->d_adjsrc) {  // per-direction source of the RLMDG adjoint sweeps
    rc = check_hip(h, hipMalloc((void**)&h->d_adjsrc, (size_t)h->ndir * nc * sizeof(double)), "hipMalloc adjoint source");
    if (rc != LMDG_OK) return rc;
  }
  double* c = h->d_cvec;
  double* xf = h->d_cvec + N;
  double* phi = h->d_cvec + 2 * N;
  double* Lam = h->d_cvec + 3 * N;
  double* xa = h->d_cvec + 4 * N;
  double* bil = h->d_cvec + 5 * N;  // n_cells used
  const auto t_start = std::chrono::steady_clock::now();
  // forward solve
  lmdg_info inf_f{}, inf_a{};
  rc = solve_impl(h, scheme, mode, tol, restart, max_iter, nullptr, xf, phi, nullptr, &inf_f, st, nullptr, nullptr);
  double J = 0.0;
  if (rc == LMDG_OK) rc = dot(h, det, phi, N, &J, st);
  // adjoint: on a centrally symmetric quadrature L_l^T is the upwind operator of
  // -Omega_l, so A^T lambda = j is the forward system with source moments d and the
  // direction blocks exchanged l <-> -l; the same sweeps solve it
  const double* xa_rec = xa;  // the adjoint solution as the recovery sweep takes it
  if (rc == LMDG_OK && rlm) {
    // RLMDG (Petrov-Galerkin): the transposed system is a scheme of its own, solved by the
    // same GMRES with the adjoint sweeps (adj_rlm_source_kernel); its solution X' gives the
    // adjoint scalar flux [P_0 mu ; -X'_1]
    h->adj_rlm = true;
    h->adj_det = det;
    rc = solve_impl(h, scheme, mode, tol, restart, max_iter, nullptr, xa, Lam, nullptr, &inf_a, st, nullptr, nullptr);
    h->adj_rlm = false;
  } else if (rc == LMDG_OK) {
    h->src0 = det;
    h->src1 = scheme == LMDG_SCHEME_STD ? det + nc : nullptr;
    const double* rhs_x = nullptr;
    const double* cshift = nullptr;
    if (scheme == LMDG_SCHEME_LMDG) {
      // Step 1: c = B_11^{-1} Sigma Q_1 (Sigma Q_1 = d_1 since sum_l w_l = 1)
      rc = cg_b11(h, det, c, std::min(1e-13, 1e-3 * tol), st);
      if (rc == LMDG_OK) {
        double* t = h->ws.vec + 3 * N;
        lmdg::vec_axpby(t, -1.0, c, 0.0, N, st);
        rhs_x = t;
        cshift = c;
      }
    }
    if (rc == LMDG_OK)
      rc = solve_impl(h, scheme, mode, tol, restart, max_iter, nullptr, xa, Lam, nullptr, &inf_a, st, rhs_x, cshift);
    if (rc == LMDG_OK && cshift) {
      double* t = h->ws.vec + 3 * N;  // x - c, the vector the recovery sweep takes
      lmdg::vec_copy(t, xa, N, st);
      lmdg::vec_axpby(t, -1.0, cshift, 1.0, N, st);
      xa_rec = t;
    }
    h->src0 = nullptr;
    h->src1 = nullptr;
  }
  // gradients: per quadrant, recompute the forward fluxes of its directions and the
  // adjoint-type fluxes of the opposite quadrant, and accumulate the angular sum
  if (rc == LMDG_OK) {
    lmdg::vec_fill(bil, 0.0, nc, st);
    for (int q = 0; q < 4 && rc == LMDG_OK; ++q) {
      rc = lmdg::launch_sweep(h, scheme, LMDG_PREC_FP64, xf, true, h->d_psi_f, st, false, 1 << q, true);
      if (rc != LMDG_OK) break;
      if (rlm) {
        // adjoint cell constants mu of the opposite quadrant (the reflected directions)
        h->adj_rlm = true;
        h->adj_det = det;
        lmdg::launch_adj_rlm_source(h, xa, det, st);
        rc = lmdg::launch_sweep(h, scheme, LMDG_PREC_FP64, nullptr, false, h->d_psi_a, st, false, 1 << (q ^ 3), true);
        h->adj_rlm = false;
        if (rc == LMDG_OK) lmdg::launch_grad_accumulate(h, q, npsi, bil, st);
        continue;
      }
      h->src0 = det;
      h->src1 = scheme == LMDG_SCHEME_STD ? det + nc : nullptr;
      rc = lmdg::launch_sweep(h, scheme, LMDG_PREC_FP64, xa_rec, true, h->d_psi_a, st, false, 1 << (q ^ 3), true);
      h->src0 = nullptr;
      h->src1 = nullptr;
      if (rc == LMDG_OK) lmdg::launch_grad_accumulate(h, q, npsi, bil, st);
    }
  }
  if (rc == LMDG_OK) {
    lmdg::launch_gradients(h, npsi, bil, phi, Lam, g_sigma_s, g_sigma_a, g_q, st);
    rc = check_hip(h, hipGetLastError(), "gradients");
  }
  if (rc == LMDG_OK) rc = check_hip(h, hipStreamSynchronize(st), "adjoint");
  if (rc == LMDG_OK) rc = read_error_flag(h, st);
  *J_out = J;
  if (info) {
    info->iterations = inf_f.iterations + inf_a.iterations;
    info->restarts = inf_f.restarts + inf_a.restarts;
    info->ir_passes = inf_f.ir_passes + inf_a.ir_passes;
    info->converged = (inf_f.converged && inf_a.converged) ? 1 : 0;
    info->rel_residual = std::max(inf_f.rel_residual, inf_a.rel_residual);
    info->time_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    info->time_apply_ms = inf_f.time_apply_ms + inf_a.time_apply_ms;
  }
  return rc;
}

int lmdg_workspace_bytes(const lmdg_t* h, int restart, int64_t* held, int64_t* solve) {
  using namespace lmdg;
  if (!h || !held || !solve || restart < 1 || restart > kMaxRestart) return LMDG_INVALID_ARG;
  const long long nc = h->ncell;
  const size_t d = sizeof(double);
  const size_t nr = (size_t)h->rhs_cap;
  size_t b = (size_t)h->noct * h->dslots * kDirStride * d + sizeof(unsigned int) + sizeof(int) +
             (size_t)h->noct * h->dslots * 2 * d;
  b += nr * (h->ws.part_bytes + std::max<size_t>(h->ws.edge_bytes, 8) + h->ws.zbuf_bytes +
             h->ws.prog_words * sizeof(unsigned long long) + (size_t)kScratchVecs * h->np * nc * d + nc * d);
  if (h->have_mat) b += 4 * (size_t)nc * d;  // sigma_t, scattering, absorption, eps (the source is above)
  if (h->d_qS) b += 3 * (size_t)nc * d;
  if (h->d_qdir) b += (size_t)h->ndir * 4 * nc * d;
  if (h->d_sq1) b += 3 * (size_t)nc * d;
  if (h->d_alpha) b += (size_t)h->ndir * (h->n[0] + h->n[1]) * 3 * d;
  if (h->d_sqa) b += 3 * (size_t)nc * d;
  b += h->krylov_doubles * d + h->small_doubles * d + 2 * h->psi_doubles * d;
  if (h->d_cvec) b += 6 * (size_t)h->np * nc * d;
  b += lmdg::pc_bytes(h);
  *held = (int64_t)b;
  // what a solve with this restart (and the handle's augmentation) allocates beyond that
  const int ka = std::max(0, std::min(h->augment, kMaxRestart - restart));
  const long long NT = (long long)h->np * nc * h->n_rhs;
  const bool pcs = h->pc_kind != LMDG_PRECOND_NONE;
  const size_t kry = std::max(krylov_doubles(restart + ka, ka, pcs, false, NT),   // FP64 solves
                              krylov_doubles(restart + ka, ka, pcs, true, NT));   // inner solves of MIXED
  const size_t small = small_layout(h->n_rhs).total;
  *solve = (int64_t)((kry > h->krylov_doubles ? kry : 0) + (small > h->small_doubles ? small : 0)) * (int64_t)d;
  return LMDG_OK;
}

int lmdg_synchronize(lmdg_t* h, void* stream) {
  if (!h) return LMDG_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  int rc = check_hip(h, hipStreamSynchronize(st), "synchronize");
  if (rc == LMDG_OK) rc = read_error_flag(h, st);
  return rc;
}

int lmdg_set_wait_limit(lmdg_t* h, long long spins, int unreachable) {
  if (!h) return LMDG_INVALID_ARG;
  if (spins < 1 || (unreachable != 0 && unreachable != 1))
    return set_error(h, LMDG_INVALID_ARG, "wait limit out of range");
  h->spin_limit = spins;
  h->wait_bias = (unsigned)unreachable;
  return LMDG_OK;
}

int lmdg_set_reconstruction(lmdg_t* h, int stencil, int suppress) {
  if (!h) return LMDG_INVALID_ARG;
  if ((stencil != 2 && stencil != 3) || (suppress != 0 && suppress != 1))
    return set_error(h, LMDG_INVALID_ARG, "stencil must be 2 or 3 and suppress 0 or 1");
  const int flags = (stencil == 3 ? 1 : 0) | (suppress ? 2 : 0);
  if (flags && h->dim != 2) return set_error(h, LMDG_UNSUPPORTED, "reconstruction variants on 3D meshes");
  h->recon_flags = flags;
  return LMDG_OK;
}

int lmdg_set_augment(lmdg_t* h, int k) {
  if (!h) return LMDG_INVALID_ARG;
  if (k < 0 || k > kMaxRestart - 1) return set_error(h, LMDG_INVALID_ARG, "augmentation count out of range");
  h->augment = k;
  return LMDG_OK;
}

int lmdg_set_refinement(lmdg_t* h, double inner_tol) {
  if (!h) return LMDG_INVALID_ARG;
  if (!(inner_tol >= 1e-6 && inner_tol <= 0.5)) return set_error(h, LMDG_INVALID_ARG, "inner tolerance out of range");
  h->ir_inner = inner_tol;
  return LMDG_OK;
}

int lmdg_set_preconditioner(lmdg_t* h, int kind, int cycles) {
  if (!h) return LMDG_INVALID_ARG;
  if (kind < LMDG_PRECOND_NONE || kind > LMDG_PRECOND_TWO_LEVEL || cycles < 1 || cycles > 50)
    return set_error(h, LMDG_INVALID_ARG, "preconditioner kind or cycles out of range");
  if (kind != LMDG_PRECOND_NONE && (h->dim != 2 || h->slab))
    return set_error(h, LMDG_UNSUPPORTED, "the preconditioner is built for 2D handles");
  h->pc_kind = kind;
  h->pc_cycles = cycles;
  return LMDG_OK;
}

int lmdg_precond_apply(lmdg_t* h, int scheme, const double* r, double* z, void* stream) {
  int rc = check_call(h, scheme, LMDG_PREC_FP64);
  if (rc != LMDG_OK) return rc;
  if (!r || !z) return set_error(h, LMDG_INVALID_ARG, "NULL vector");
  hipStream_t st = (hipStream_t)stream;
  if (h->pc_kind == LMDG_PRECOND_NONE) {
    lmdg::vec_copy(z, r, (long long)h->np * h->ncell * h->n_rhs, st);
    return check_hip(h, hipGetLastError(), "copy");
  }
  return lmdg::pc_apply(h, scheme, r, z, st);
}

int lmdg_profile(lmdg_t* h, int enable) {
  if (!h) return LMDG_INVALID_ARG;
  h->profiling = enable != 0;
  h->ev_used = 0;
  return LMDG_OK;
}

int lmdg_sweep_kernel_time(lmdg_t* h, double* total_ms, int* launches) {
  if (!h || !total_ms || !launches) return LMDG_INVALID_ARG;
  double total = 0;
  for (size_t k = 0; k + 1 < h->ev_used; k += 2) {
    int rc = check_hip(h, hipEventSynchronize(h->ev_pool[k + 1]), "event sync");
    if (rc != LMDG_OK) return rc;
    float ms = 0;
    rc = check_hip(h, hipEventElapsedTime(&ms, h->ev_pool[k], h->ev_pool[k + 1]), "event time");
    if (rc != LMDG_OK) return rc;
    total += ms;
  }
  *total_ms = total;
  *launches = (int)(h->ev_used / 2);
  h->ev_used = 0;
  return LMDG_OK;
}

}  // extern "C"
