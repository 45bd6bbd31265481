// K x without allocation: the sweep workspace of lmdg_apply (quadrant partials, edge
// traces, 3D per-cell coefficients, progress words, ticket counter and error flag) taken from a
// fixed device array instead of the handle's buffers, for callers that cannot allocate.
#include <mutex>

#include "internal.h"

namespace lmdg {
namespace {

// Fixed sweep workspace, one copy per GPU the library runs on (held until the process
// ends).  Host code never uses this name as an address: scratch_ptr() below holds the
// device address of each GPU's copy.
constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_ptr[kMaxDevices] = {};

// Device address of the current GPU's copy (looked up once per device).
int scratch_ptr(lmdg_handle* h, int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return set_error(h, LMDG_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const int rc = check_hip(h, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (rc != LMDG_OK) return rc;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return LMDG_OK;
}

// Zero n 64-bit words (progress words, ticket and flag) with a plain kernel.
__global__ void clear_words_kernel(unsigned long long* __restrict__ w, long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    w[e] = 0ull;
}

// Carry a failed wait of the fixed workspace over to the handle's own sticky flag,
// which the synchronising calls report.
__global__ void merge_flag_kernel(const int* __restrict__ from, int* __restrict__ to) {
  if (threadIdx.x == 0 && *from) atomicOr(to, 1);
}

inline size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

int apply_op_impl(lmdg_handle* h, int scheme, int prec, const double* x, double* y, hipStream_t st);  // api.cpp

}  // namespace lmdg

extern "C" int lmdg_apply_noalloc(lmdg_t* h, int scheme, int prec, const double* x, double* y, void* stream) {
  using namespace lmdg;
  if (!h) return LMDG_INVALID_ARG;
  if (!x || !y) return set_error(h, LMDG_INVALID_ARG, "NULL vector");
  if (scheme < LMDG_SCHEME_STD || scheme > LMDG_SCHEME_RLMDG) return set_error(h, LMDG_INVALID_ARG, "unknown scheme");
  if (prec != LMDG_PREC_FP64 && prec != LMDG_PREC_FP32) return set_error(h, LMDG_INVALID_ARG, "unknown precision");
  if (!h->have_mat) return set_error(h, LMDG_INVALID_ARG, "materials not set");
  int dev = -1;
  int rc = check_hip(h, hipGetDevice(&dev), "hipGetDevice");
  if (rc != LMDG_OK) return rc;
  if (dev != h->device) return set_error(h, LMDG_INVALID_ARG, "the handle's device is not the current device");
  // layout: flags (ticket, error flag) | progress words | edge traces | 3D coefficients | partials
  const size_t nr = (size_t)h->n_rhs;
  const size_t flags = 256;
  const size_t prog = round256(h->ws.prog_words * nr * sizeof(unsigned long long));
  const size_t edge = round256(std::max<size_t>(h->ws.edge_bytes * nr, 8));
  const size_t zbuf = round256(h->ws.zbuf_bytes * nr);
  const size_t part = round256(h->ws.part_bytes * nr);
  const size_t need = flags + prog + edge + zbuf + part;
  if (need > kScratchBytes)
    return set_error(h, LMDG_INVALID_ARG,
                     "workspace of " + std::to_string(need) + " bytes exceeds the fixed " +
                         std::to_string(kScratchBytes) + "-byte array of lmdg_apply_noalloc");
  void* base = nullptr;
  rc = scratch_ptr(h, dev, &base);
  if (rc != LMDG_OK) return rc;
  unsigned char* b = static_cast<unsigned char*>(base);
  hipStream_t st = (hipStream_t)stream;
  // every call starts from cleared flags, ticket and progress words: the array keeps the
  // last call's contents, possibly of another handle with other epochs
  const long long words = (long long)((flags + prog) / 8);
  hipLaunchKernelGGL(clear_words_kernel, dim3((unsigned)std::min<long long>((words + 255) / 256, 1024)), dim3(256), 0,
                     st, reinterpret_cast<unsigned long long*>(b), words);
  rc = check_hip(h, hipGetLastError(), "clear fixed workspace");
  if (rc != LMDG_OK) return rc;
  Workspace saved = h->ws;
  const unsigned int saved_ticket = h->ticket_base;
  const bool saved_prof = h->profiling;
  h->ws.ticket = reinterpret_cast<unsigned int*>(b);
  h->ws.err = reinterpret_cast<int*>(b + 8);
  h->ws.prog = reinterpret_cast<unsigned long long*>(b + flags);
  h->ws.edge = b + flags + prog;
  h->ws.zbuf = h->ws.zbuf_bytes ? b + flags + prog + edge : nullptr;
  h->ws.part = reinterpret_cast<double*>(b + flags + prog + edge + zbuf);
  h->ticket_base = 0;
  h->profiling = false;  // no event recording (it may create events)
  rc = apply_op_impl(h, scheme, prec, x, y, st);
  if (rc == LMDG_OK) {
    hipLaunchKernelGGL(merge_flag_kernel, dim3(1), dim3(64), 0, st, (const int*)(b + 8), saved.err);
    rc = check_hip(h, hipGetLastError(), "merge flag");
  }
  h->ws = saved;
  h->ticket_base = saved_ticket;
  h->profiling = saved_prof;
  return rc;
}
