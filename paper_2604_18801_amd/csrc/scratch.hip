// Allocation-free friends-of-friends labels: the same cell build, pair pass
// and union-find as pcc_fof_labels, with every device buffer carved from one
// static device array instead of the context's workspace arena.
//
// Each GPU holds its own copy of the array (from the library's first use of
// that GPU until the process ends).  Its device address is looked up once
// per device, when the first context on that device is created; host code
// only ever passes that address, never the array's name, to kernels.
#include <atomic>
#include <cstring>
#include <mutex>
#include <string>

#include "host.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)128 << 20;
// The labels-only path takes at most ~240 bytes per particle from its arena
// (inputs copied from the host 24, cell keys and sort 48, sorted positions
// 32, cell tables 86 (starts, keys, cell of each particle, nine neighbour
// ranges, face bits, coarse key index), pair plan 37, union-finds and
// counts 24, labels 8), plus a few kB of per-call tables and 256-byte
// rounding: 256 per particle and 1 MiB bound it.
constexpr size_t kBytesPerParticle = 256;
constexpr size_t kFixedBytes = (size_t)1 << 20;
constexpr int64_t kMaxParticles = (int64_t)((kScratchBytes - kFixedBytes) / kBytesPerParticle);
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_init_mu;
void *g_ptr[kMaxDevices] = {};         // device address of `scratch` per device
std::mutex g_call_mu[kMaxDevices];     // one call at a time per device
std::atomic<int64_t> g_high_water{0};  // arena bytes the last call used

pcc_status fail(pcc_status s, const std::string &m) {
  pcc::set_last_error(m);
  return s;
}

}  // namespace

namespace pcc {

void scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices)
    throw Error(PCC_E_UNSUPPORTED, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> g(g_init_mu);
  if (g_ptr[device]) return;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Error(PCC_E_DEVICE, std::string("hipGetSymbolAddress of the static scratch failed: ") +
                                  hipGetErrorString(e));
  }
  g_ptr[device] = p;
}

int64_t noalloc_high_water() { return g_high_water.load(); }

}  // namespace pcc

extern "C" {

int64_t pcc_fof_labels_noalloc_max_n(void) { return kMaxParticles; }

pcc_status pcc_fof_labels_noalloc(pcc_context *ctx, const pcc_particles *pts, double b,
                                  const double box[3], int32_t *labels, void *hip_stream) {
  if (!ctx || !pts || !labels) return fail(PCC_E_INVALID_ARG, "NULL argument");
  if (pts->n < 0) return fail(PCC_E_INVALID_ARG, "n < 0");
  if (pts->n > kMaxParticles)
    return fail(PCC_E_INVALID_ARG,
                "n = " + std::to_string(pts->n) + " exceeds the static scratch limit of " +
                    std::to_string(kMaxParticles) + " particles (pcc_fof_labels has no limit)");
  const int dev = ctx->c.device;
  if (dev < 0 || dev >= kMaxDevices || !g_ptr[dev])
    return fail(PCC_E_DEVICE, "no static scratch address for this device");
  try {
    pcc::set_last_error("");
    std::lock_guard<std::mutex> g(g_call_mu[dev]);
    pcc::Arena ar;
    ar.attach(g_ptr[dev], kScratchBytes);
    pcc_job job;
    std::memset(&job, 0, sizeof job);
    job.orig = *pts;
    job.recon = *pts;
    pcc_params_init(&job.params);
    job.params.b = b;
    job.params.xi = 0.0;
    if (box)
      for (int a = 0; a < 3; ++a) job.params.box[a] = box[a];
    job.out.labels = labels;
    pcc_job_result r;
    std::memset(&r, 0, sizeof r);
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->c.own;
    pcc::run_batch(ctx->c, &job, 1, &r, s, true, false, &ar);
    g_high_water.store((int64_t)ar.high_water());
    if (r.status < 0) return fail(r.status, pcc_status_string(r.status));
    return PCC_OK;
  } catch (const pcc::Error &e) {
    return fail(e.status, e.what());
  } catch (const std::exception &e) {
    return fail(PCC_E_DEVICE, e.what());
  }
}

}  // extern "C"
