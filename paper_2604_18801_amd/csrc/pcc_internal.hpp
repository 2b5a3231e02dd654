// Internal declarations of the gfx950 correction library.
//
// All jobs of one call live in one global index space: job k owns particles
// [p_off[k], p_off[k+1]) of every particle array, the cells
// [cell_base[k], cell_base[k] + ncell[k]) of the cell grid, and a contiguous
// range of editable rows.  A plain call is a batch of one job.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <atomic>
#include <vector>

namespace pcc {

constexpr int kWave = 64;

struct Error : std::runtime_error {
  int status;
  Error(int s, const std::string &m) : std::runtime_error(m), status(s) {}
};

void hip_fail(hipError_t e, const char *what, const char *file, int line);
#define PCC_HIP(call)                                          \
  do {                                                         \
    hipError_t e_ = (call);                                    \
    if (e_ != hipSuccess) ::pcc::hip_fail(e_, #call, __FILE__, __LINE__); \
  } while (0)

// Per-job constants read by the kernels (one entry per job, device memory).
// linking lengths of one multi-threshold correction, at most
constexpr int kMaxThresholds = 8;
// column word of an incidence: partner row | threshold index << 28 | pc bit
constexpr uint32_t kColRow = 0x0fffffffu;
constexpr int kColThrShift = 28;
constexpr uint32_t kColPc = 0x80000000u;

struct JobDev {
  int64_t p_off;        // first particle of the job in the global arrays
  int64_t n;            // particles
  // pair predicates, squared distances in float64 (Sec. 3.1, 3.2)
  double rs2, b2, rv2;  // rs2 < 0 when b - 2 sqrt(3) xi <= 0 (no safe links)
  // float32 classification bands of the three thresholds: a float32 d^2
  // below *_lo (above *_hi) is below (above) the threshold in the exact
  // float64 predicate; in between, the float64 predicate decides
  float f_rs_lo, f_rs_hi, f_b_lo, f_b_hi, f_rv_lo;
  float rv2_f32;        // f_rv_hi: conservative float32 prefilter of d^2 <= rv2
  // every periodic coordinate of the originals lies in [0, L): a partner's
  // periodic image is fixed per neighbour cell (cell edge bits), and no
  // candidate needs the per-pair minimum-image wrap
  int32_t img;
  int32_t mode;
  // periodic axes: side and half side (half = +inf on open axes)
  double L[3], hL[3];
  float Lf[3], hLf[3];
  // cell grid (Sec. 2.4.1, 3.3): cells of side >= r_v
  double origin[3], inv_w[3];
  int32_t nc[3];
  int32_t periodic;     // bit a set when axis a is periodic
  uint32_t cell_base;   // first cell key of the job
  // correction loop (Alg. 1, Eq. 3, Sec. 4.2)
  double b, bm, bp, bm2, bp2;  // b -+ delta_t
  double xi_p;                 // box half width
  double lr, beta1, beta2, adam_eps, one_m_beta1, one_m_beta2;
  // [t] = (1 - beta1^t, 1 - beta2^t) for t = 0 .. bc_len - 1; the last entry
  // also stands for every later t (both corrections have reached 1 exactly,
  // or the table covers t = max_iters + 1)
  const double2 *bc_tab;
  int64_t bc_len;
  int64_t max_iters;
  double loss_tol;
  int32_t optimizer;
  int32_t m_bits;
  // quantiser of the edits
  double qstep, qoffset;       // edit = code * qstep - qoffset
  double qmax;                 // 2^m - 1
  // tightened bounds b_k -+ delta_t of every linking length of a
  // multi-threshold correction (entry 0 = this job's own b); an incidence's
  // threshold index sits in its column word
  int32_t nthr;
  double thr_bm[kMaxThresholds], thr_bp[kMaxThresholds];
  double thr_bm2[kMaxThresholds], thr_bp2[kMaxThresholds];
  // per-evaluation trace of the loop (loss of Eq. 3, violated constraints),
  // entries 0 .. trace_cap - 1 (device; none when trace_cap = 0)
  double *trace_loss;
  unsigned long long *trace_viol;
  int64_t trace_cap;
};

// Mutable per-job state of the correction loop (device memory).
struct JobLoop {
  int64_t t;              // gradient steps applied
  int32_t done;
  int32_t status;         // 0 converged, 1 cap reached
  double bc1, bc2;        // 1 - beta^t for the next step
  unsigned long long viol0, viol_last;
  double loss0, loss_last;  // tightened loss of Eq. 3, float64
  unsigned long long rows_eval, inc_eval;  // rows and incidences evaluated, all steps
  int32_t have0;
  int32_t pad;
};

// Device helper: the job that owns global index g, by binary search in
// off[0..njobs] (off[njobs] = total).
__device__ inline int job_of(const int64_t *__restrict__ off, int njobs, int64_t g) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Device memory arena: grow-only chunks, reset per call; after the first
// call of a given size the steady state allocates nothing.
// ---------------------------------------------------------------------------
// Test hook (pcc_debug_set): when >= 0, the number of further arena
// allocations that succeed before one fails as if the device were out of
// memory; -1 when off.  Process-wide.
extern std::atomic<int64_t> g_alloc_fail_after;

class Arena {
 public:
  ~Arena();
  void *alloc(size_t bytes);
  template <typename T>
  T *get(size_t count) {
    return static_cast<T *>(alloc(count * sizeof(T)));
  }
  void reset();          // start a new call (previous data becomes invalid)
  void release();        // free everything
  // Serve every request from the caller's buffer [base, base + bytes) and
  // never allocate: a request that does not fit throws PCC_E_OUT_OF_MEMORY.
  // release() then forgets the buffer without freeing it.
  void attach(void *base, size_t bytes);
  size_t used() const { return used_; }
  size_t capacity() const {  // device bytes the arena holds
    size_t c = 0;
    for (const auto &k : chunks_) c += k.size;
    return c;
  }
  size_t high_water() const { return high_; }  // most bytes in use since reset()
  bool fixed() const { return fixed_; }  // serving from a borrowed buffer
  size_t spare() const {  // held bytes not yet handed out in this call
    size_t c = 0;
    for (const auto &k : chunks_) c += k.size - k.off;
    return c;
  }

 private:
  struct Chunk {
    char *base;
    size_t size, off;
  };
  std::vector<Chunk> chunks_;
  size_t used_ = 0, high_ = 0, last_total_ = 0;
  bool fixed_ = false;  // chunks_ holds one borrowed buffer
};

// ---------------------------------------------------------------------------
// primitives (prims.hip)
// ---------------------------------------------------------------------------
// exclusive prefix sums; `out` may alias `in` only for equal types.
// If total != nullptr, *total (device) receives the sum of all inputs.
void scan_u32_u64(const uint32_t *in, uint64_t *out, size_t n, uint64_t *total,
                  Arena &ar, hipStream_t s);
void scan_u8_u32(const uint8_t *in, uint32_t *out, size_t n, uint32_t *total,
                 Arena &ar, hipStream_t s);
void scan_u32_u32(const uint32_t *in, uint32_t *out, size_t n, uint32_t *total,
                  Arena &ar, hipStream_t s);
// exclusive scans; `out` may be `in`
void scan_u64_u64(const uint64_t *in, uint64_t *out, size_t n, uint64_t *total,
                  Arena &ar, hipStream_t s);
// stable LSD radix sort of (key, value) on the low `bits` bits of the keys;
// results land in keys/vals (tmp buffers from the arena).
void radix_sort_u32(uint32_t *keys, uint32_t *vals, size_t n, int bits, Arena &ar,
                    hipStream_t s);
void fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
void fill_u64(uint64_t *p, uint64_t v, size_t n, hipStream_t s);
void fill_u8(uint8_t *p, uint8_t v, size_t n, hipStream_t s);
void iota_u32(uint32_t *p, size_t n, hipStream_t s);

inline int blocks_for(size_t n, int threads, int cap = 1 << 20) {
  size_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > (size_t)cap) b = cap;
  return (int)b;
}

}  // namespace pcc
