// C ABI of include/pcc.h: argument checks, context management, error
// reporting; every entry point catches all exceptions at this boundary.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "host.hpp"

namespace {
thread_local std::string g_err;

pcc_status fail(pcc_status s, const std::string &m) {
  g_err = m;
  return s;
}

template <typename F>
pcc_status guarded(F &&f) {
  try {
    g_err.clear();
    return f();
  } catch (const pcc::Error &e) {
    return fail(e.status, e.what());
  } catch (const std::bad_alloc &) {
    return fail(PCC_E_OUT_OF_MEMORY, "host allocation failed");
  } catch (const std::exception &e) {
    return fail(PCC_E_DEVICE, e.what());
  }
}

hipStream_t pick(pcc_context *ctx, void *s) {
  return s ? (hipStream_t)s : ctx->c.own;
}
}  // namespace

extern "C" {

int pcc_version(void) { return PCC_VERSION; }

const char *pcc_status_string(pcc_status s) {
  switch (s) {
    case PCC_OK: return "ok";
    case PCC_NOT_CONVERGED: return "not converged (iteration cap reached)";
    case PCC_PENDING: return "pending";
    case PCC_E_INVALID_ARG: return "invalid argument";
    case PCC_E_OUT_OF_MEMORY: return "out of memory";
    case PCC_E_DEVICE: return "device error";
    case PCC_E_BUFFER_TOO_SMALL: return "buffer too small";
    case PCC_E_INPUT_BOUND: return "reconstruction outside the error bound";
    case PCC_E_UNSUPPORTED: return "unsupported";
    case PCC_E_CANCELLED: return "cancelled";
    default: return "unknown status";
  }
}

const char *pcc_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace pcc {
void set_last_error(const std::string &m) { g_err = m; }
}  // namespace pcc

extern "C" {

pcc_status pcc_context_set(pcc_context *ctx, int32_t key, int64_t value) {
  if (!ctx) return fail(PCC_E_INVALID_ARG, "NULL context");
  if (key == PCC_CTX_KERNEL_TIMING) {
    if (value != 0 && value != 1) return fail(PCC_E_INVALID_ARG, "kernel timing is 0 or 1");
    ctx->c.kt.on = value != 0;
    return PCC_OK;
  }
  if (key == PCC_CTX_GRAPH_ITERS) {
    if (value < 1 || value > 64) return fail(PCC_E_INVALID_ARG, "graph iterations lie in 1..64");
    ctx->c.graph_iters = (int)value;
    return PCC_OK;
  }
  if (key == PCC_CTX_EXACT_PAIRS) {
    if (value != 0 && value != 1) return fail(PCC_E_INVALID_ARG, "exact pairs is 0 or 1");
    ctx->c.force_exact_pairs = value != 0;
    return PCC_OK;
  }
  if (key == PCC_CTX_CELL_PCT) {
    if (value < 100 || value > 400) return fail(PCC_E_INVALID_ARG, "cell side lies in 100..400 %");
    ctx->c.cell_pct = (int)value;
    return PCC_OK;
  }
  if (key == PCC_CTX_DENSE_CELL) {
    if (value < 1 || value > 4096) return fail(PCC_E_INVALID_ARG, "dense-cell threshold lies in 1..4096");
    ctx->c.dense_cell = (int)value;
    return PCC_OK;
  }
  return fail(PCC_E_INVALID_ARG, "unknown context option");
}

pcc_status pcc_context_get(pcc_context *ctx, int32_t key, int64_t *value) {
  if (!ctx || !value) return fail(PCC_E_INVALID_ARG, "NULL argument");
  switch (key) {
    case PCC_CTX_KERNEL_TIMING: *value = ctx->c.kt.on ? 1 : 0; return PCC_OK;
    case PCC_CTX_GRAPH_ITERS: *value = ctx->c.graph_iters; return PCC_OK;
    case PCC_CTX_EXACT_PAIRS: *value = ctx->c.force_exact_pairs ? 1 : 0; return PCC_OK;
    case PCC_CTX_CELL_PCT: *value = ctx->c.cell_pct; return PCC_OK;
    case PCC_CTX_DENSE_CELL: *value = ctx->c.dense_cell; return PCC_OK;
    case PCC_CTX_WORKSPACE_HIGH_WATER: *value = (int64_t)ctx->c.arena.high_water(); return PCC_OK;
    default: return fail(PCC_E_INVALID_ARG, "unknown context option");
  }
}

pcc_status pcc_debug_set(int32_t key, int64_t value) {
  if (key != PCC_DEBUG_ALLOC_FAIL_AFTER) return fail(PCC_E_INVALID_ARG, "unknown debug key");
  if (value < -1) return fail(PCC_E_INVALID_ARG, "value must be >= -1");
  pcc::g_alloc_fail_after.store(value);
  return PCC_OK;
}

pcc_status pcc_debug_get(int32_t key, int64_t *value) {
  if (!value) return fail(PCC_E_INVALID_ARG, "bad argument");
  if (key == PCC_DEBUG_ALLOC_FAIL_AFTER) {
    *value = pcc::g_alloc_fail_after.load();
    return PCC_OK;
  }
  if (key == PCC_DEBUG_NOALLOC_HIGH_WATER) {
    *value = pcc::noalloc_high_water();
    return PCC_OK;
  }
  return fail(PCC_E_INVALID_ARG, "unknown debug key");
}

pcc_status pcc_autotune(pcc_context *ctx, const pcc_job *jobs, int32_t njobs, int32_t flags,
                        pcc_tune_report *rep, void *hip_stream) {
  if (!ctx || njobs < 1 || !jobs) return fail(PCC_E_INVALID_ARG, "NULL argument or no job");
  return guarded([&]() -> pcc_status {
    pcc_tune_report r;
    pcc::autotune(ctx->c, jobs, njobs, pick(ctx, hip_stream), flags, r);
    if (rep) *rep = r;
    return PCC_OK;
  });
}

void pcc_params_init(pcc_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->mode = PCC_MODE_HF;
  p->m_bits = 16;
  p->optimizer = PCC_OPT_ADAM;
  p->margin_policy = PCC_MARGIN_SAFE;
  p->lr = 1e-3;
  p->beta1 = 0.9;
  p->beta2 = 0.999;
  p->adam_eps = 1e-8;
  p->max_iters = 0;
  p->loss_tol = 0.0;
}

size_t pcc_stream_bound(int64_t n, const pcc_params *p) {
  return pcc::stream_bound(n, p ? p->m_bits : 16);
}

pcc_status pcc_context_create(int device, pcc_context **out) {
  if (!out) return fail(PCC_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  return guarded([&]() -> pcc_status {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0)
      return fail(PCC_E_DEVICE, "no HIP device is visible");
    if (device < 0 || device >= count) return fail(PCC_E_INVALID_ARG, "device index out of range");
    PCC_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    PCC_HIP(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      return fail(PCC_E_UNSUPPORTED, std::string("built for gfx950, device is ") + prop.gcnArchName);
    // the device's static scratch of the allocation-free calls
    pcc::scratch_init(device);
    auto *c = new pcc_context;
    c->c.device = device;
    if (hipStreamCreate(&c->c.own) != hipSuccess) {
      delete c;
      return fail(PCC_E_DEVICE, "hipStreamCreate failed");
    }
    try {
      pcc::create_events(c->c);
    } catch (...) {
      for (auto &e : c->c.ev)
        if (e) hipEventDestroy(e);
      hipStreamDestroy(c->c.own);
      delete c;
      throw;
    }
    *out = c;
    return PCC_OK;
  });
}

pcc_status pcc_context_destroy(pcc_context *ctx) {
  if (!ctx) return PCC_OK;
  hipSetDevice(ctx->c.device);
  hipDeviceSynchronize();
  ctx->c.pgd_graph.clear();
  ctx->c.arena.release();
  for (auto &t : ctx->c.bc) hipFree(t.dev);
  for (auto &e : ctx->c.ev)
    if (e) hipEventDestroy(e);
  if (ctx->c.pinned) hipHostFree(ctx->c.pinned);
  if (ctx->c.own) hipStreamDestroy(ctx->c.own);
  delete ctx;
  return PCC_OK;
}

pcc_status pcc_correct(pcc_context *ctx, const pcc_particles *orig, const pcc_particles *recon,
                       const pcc_params *params, pcc_outputs *out, pcc_stats *stats,
                       void *hip_stream) {
  if (!ctx || !orig || !recon || !params || !out)
    return fail(PCC_E_INVALID_ARG, "NULL argument");
  return guarded([&]() -> pcc_status {
    pcc_job job;
    job.orig = *orig;
    job.recon = *recon;
    job.params = *params;
    job.out = *out;
    pcc_job_result r;
    std::memset(&r, 0, sizeof r);
    pcc::run_batch(ctx->c, &job, 1, &r, pick(ctx, hip_stream), false);
    if (stats) *stats = r.stats;
    if (r.status < 0 && g_err.empty()) g_err = pcc_status_string(r.status);
    return r.status;
  });
}

pcc_status pcc_workspace_query(pcc_context *ctx, const pcc_particles *orig,
                               const pcc_particles *recon, const pcc_params *params,
                               size_t *bytes, void *hip_stream) {
  if (!ctx || !orig || !recon || !params || !bytes)
    return fail(PCC_E_INVALID_ARG, "NULL argument");
  *bytes = 0;
  return guarded([&]() -> pcc_status {
    pcc_job job;
    std::memset(&job, 0, sizeof job);
    job.orig = *orig;
    job.recon = *recon;
    job.params = *params;
    pcc_job_result r;
    std::memset(&r, 0, sizeof r);
    size_t fp = 0;
    pcc::run_batch(ctx->c, &job, 1, &r, pick(ctx, hip_stream), false, false, nullptr, &fp);
    if (r.status < 0) {
      if (g_err.empty()) g_err = pcc_status_string(r.status);
      return r.status;
    }
    *bytes = fp;
    return PCC_OK;
  });
}

pcc_status pcc_correct_multi(pcc_context *ctx, const pcc_particles *orig,
                             const pcc_particles *recon, const pcc_params *params,
                             const double *b_list, int32_t nb, pcc_outputs *out, pcc_stats *stats,
                             void *hip_stream) {
  if (!ctx || !orig || !recon || !params || !out || !b_list)
    return fail(PCC_E_INVALID_ARG, "NULL argument");
  if (nb < 1 || nb > PCC_MAX_THRESHOLDS)
    return fail(PCC_E_INVALID_ARG, "the number of linking lengths must be 1 .. 8");
  for (int32_t k = 0; k < nb; ++k)
    if (!(b_list[k] > 0.0) || !std::isfinite(b_list[k]))
      return fail(PCC_E_INVALID_ARG, "every linking length must be finite and > 0");
  return guarded([&]() -> pcc_status {
    std::vector<pcc_job> jobs(nb);
    for (int32_t k = 0; k < nb; ++k) {
      pcc_job &j = jobs[k];
      j.orig = *orig;
      j.recon = *recon;
      j.params = *params;
      j.params.b = b_list[k];
      std::memset(&j.out, 0, sizeof j.out);
      if (out->labels) j.out.labels = out->labels + (size_t)k * (size_t)(orig->n > 0 ? orig->n : 0);
    }
    // job 0 carries the corrected particles: its stream and coordinates
    jobs[0].out.stream = out->stream;
    jobs[0].out.stream_cap = out->stream_cap;
    jobs[0].out.stream_len = out->stream_len;
    jobs[0].out.debug_xyz = out->debug_xyz;
    jobs[0].out.loss_trace = out->loss_trace;
    jobs[0].out.viol_trace = out->viol_trace;
    jobs[0].out.trace_cap = out->trace_cap;
    std::vector<pcc_job_result> r(nb);
    for (auto &x : r) std::memset(&x, 0, sizeof x);
    pcc::run_batch(ctx->c, jobs.data(), nb, r.data(), pick(ctx, hip_stream), false, true);
    pcc_status st = r[0].status;
    for (int32_t k = 1; k < nb; ++k)
      if (r[k].status < 0 && st >= 0) st = r[k].status;
    if (stats) *stats = r[0].stats;
    if (st < 0 && g_err.empty()) g_err = pcc_status_string(st);
    return st;
  });
}

pcc_status pcc_correct_batch(pcc_context *ctx, const pcc_job *jobs, int32_t njobs,
                             pcc_job_result *results, void *hip_stream) {
  if (!ctx || njobs < 0 || (njobs > 0 && (!jobs || !results)))
    return fail(PCC_E_INVALID_ARG, "NULL argument");
  if (njobs > PCC_MAX_BATCH_JOBS)
    return fail(PCC_E_INVALID_ARG, "at most 65536 jobs per batched call");
  return guarded([&]() -> pcc_status {
    if (njobs == 0) return PCC_OK;
    return pcc::run_batch(ctx->c, jobs, njobs, results, pick(ctx, hip_stream), false);
  });
}

pcc_status pcc_decode(const uint8_t *stream, size_t len, const pcc_particles *recon, float *ox,
                      float *oy, float *oz) {
  if (!stream || !recon) return fail(PCC_E_INVALID_ARG, "NULL argument");
  if (recon->memspace != PCC_MEM_HOST) return fail(PCC_E_UNSUPPORTED, "decode takes host arrays");
  if (recon->n > 0 && (!recon->x || !recon->y || !recon->z || !ox || !oy || !oz))
    return fail(PCC_E_INVALID_ARG, "NULL coordinate pointer");
  return guarded([&]() -> pcc_status {
    std::string err;
    pcc_status s = pcc::decode_stream(stream, len, recon->n, recon->x, recon->y, recon->z, ox, oy,
                                      oz, err);
    if (s != PCC_OK) g_err = err;
    return s;
  });
}

pcc_status pcc_decode_device(pcc_context *ctx, const uint8_t *stream, size_t len,
                             const pcc_particles *recon, float *out_x, float *out_y, float *out_z,
                             void *hip_stream) {
  if (!ctx || !stream || !recon) return fail(PCC_E_INVALID_ARG, "NULL argument");
  if (recon->memspace != PCC_MEM_DEVICE)
    return fail(PCC_E_INVALID_ARG, "pcc_decode_device takes device arrays (pcc_decode: host)");
  if (recon->n < 0) return fail(PCC_E_INVALID_ARG, "n < 0");
  if (recon->n > 0 && (!recon->x || !recon->y || !recon->z || !out_x || !out_y || !out_z))
    return fail(PCC_E_INVALID_ARG, "NULL coordinate pointer");
  return guarded([&]() -> pcc_status {
    std::string err;
    pcc::ParsedStream ps;
    const pcc_status st = pcc::parse_stream(stream, len, recon->n, ps, err, false);
    if (st != PCC_OK) return fail(st, err);
    PCC_HIP(hipSetDevice(ctx->c.device));
    ctx->c.arena.reset();
    ctx->c.last.valid = false;  // the arena's contents of the last correction are gone
    const float *rin[3] = {recon->x, recon->y, recon->z};
    float *rout[3] = {out_x, out_y, out_z};
    if (!pcc::apply_edits_device(ps, rin, rout, ctx->c.arena, pick(ctx, hip_stream)))
      return fail(PCC_E_INVALID_ARG, "corrupt Huffman data");
    return PCC_OK;
  });
}

pcc_status pcc_fof_labels(pcc_context *ctx, const pcc_particles *pts, double b,
                          const double box[3], int32_t *labels, void *hip_stream) {
  if (!ctx || !pts || !labels) return fail(PCC_E_INVALID_ARG, "NULL argument");
  return guarded([&]() -> pcc_status {
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
    pcc::run_batch(ctx->c, &job, 1, &r, pick(ctx, hip_stream), true);
    if (r.status < 0 && g_err.empty()) g_err = pcc_status_string(r.status);
    return r.status < 0 ? r.status : PCC_OK;
  });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// test hook
// ---------------------------------------------------------------------------
namespace pcc {
namespace {
__global__ void k_dbg_pairs(const uint32_t *a_i, const uint32_t *a_j, const uint8_t *a_t,
                            const uint8_t *a_k, size_t na, const float4 *pos, const int64_t *p_off,
                            int njobs, int32_t *job, uint32_t *lo, uint32_t *hi, uint8_t *t,
                            uint8_t *k) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < na;
       p += (size_t)gridDim.x * blockDim.x) {
    const uint32_t i = __float_as_uint(pos[a_i[p]].w), j = __float_as_uint(pos[a_j[p]].w);
    job[p] = job_of(p_off, njobs, (int64_t)a_i[p]);
    lo[p] = i < j ? i : j;
    hi[p] = i < j ? j : i;
    t[p] = a_t[p];
    k[p] = a_k ? a_k[p] : 0;
  }
}
__global__ void k_dbg_safe(const uint32_t *root, const float4 *pos, size_t n, int32_t *lab_sorted_root) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x)
    atomicMin(lab_sorted_root + root[k], (int32_t)__float_as_uint(pos[k].w));
}
__global__ void k_dbg_safe2(const uint32_t *root, const float4 *pos, const int64_t *p_off, int njobs,
                            size_t n, const int32_t *minid, int32_t *out) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x) {
    const int j = job_of(p_off, njobs, (int64_t)k);
    out[p_off[j] + __float_as_uint(pos[k].w)] = minid[root[k]];
  }
}
__global__ void k_dbg_e(const uint32_t *e_list, size_t ne, const float4 *pos, const int64_t *p_off,
                        int njobs, int32_t *job, uint32_t *id) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne;
       e += (size_t)gridDim.x * blockDim.x) {
    job[e] = job_of(p_off, njobs, (int64_t)e_list[e]);
    id[e] = __float_as_uint(pos[e_list[e]].w);
  }
}
}  // namespace
}  // namespace pcc

extern "C" pcc_status pcc_debug_fetch(pcc_context *ctx, int32_t job, int32_t what, void *host_dst,
                                      int64_t cap, int64_t *count) {
  if (!ctx || !count) return fail(PCC_E_INVALID_ARG, "NULL argument");
  return guarded([&]() -> pcc_status {
    using namespace pcc;
    LastCall &L = ctx->c.last;
    if (!L.valid) return fail(PCC_E_INVALID_ARG, "no retained call");
    int q = -1;
    for (int k = 0; k < (int)L.job_index.size(); ++k)
      if (L.job_index[k] == job) q = k;
    if (q < 0) return fail(PCC_E_INVALID_ARG, "job was not part of the last call");
    hipStream_t s = ctx->c.own;
    PCC_HIP(hipSetDevice(ctx->c.device));
    Arena scratch;
    int64_t *d_poff = scratch.get<int64_t>(L.p_off.size());
    PCC_HIP(hipMemcpyAsync(d_poff, L.p_off.data(), L.p_off.size() * sizeof(int64_t),
                           hipMemcpyHostToDevice, s));
    const int64_t n_job = L.p_off[q + 1] - L.p_off[q];
    if (what == PCC_DBG_CELL_START || what == PCC_DBG_NEIGHBORS) {
      uint32_t u = 0;
      if (L.n) {
        PCC_HIP(hipMemcpyAsync(&u, L.n_cells, sizeof u, hipMemcpyDeviceToHost, s));
        PCC_HIP(hipStreamSynchronize(s));
      }
      const int64_t m = what == PCC_DBG_CELL_START ? (int64_t)u + 1 : 2 * pcc::kNbrSlots * (int64_t)u;
      *count = L.n ? m : 0;
      if (!host_dst || cap < *count || !*count) return PCC_OK;
      const void *src =
          what == PCC_DBG_CELL_START ? (const void *)L.cell_start : (const void *)L.nrange;
      PCC_HIP(hipMemcpyAsync(host_dst, src, (size_t)m * 4, hipMemcpyDeviceToHost, s));
      PCC_HIP(hipStreamSynchronize(s));
      return PCC_OK;
    }
    if (what == PCC_DBG_SAFE_LABELS) {
      *count = n_job;
      if (cap < n_job || !host_dst) return PCC_OK;
      int32_t *minid = scratch.get<int32_t>(L.n ? L.n : 1), *out = scratch.get<int32_t>(L.n ? L.n : 1);
      fill_u32((uint32_t *)minid, 0x7fffffffu, L.n, s);
      k_dbg_safe<<<blocks_for(L.n, 256, 65536), 256, 0, s>>>(L.safe_root, L.pos, L.n, minid);
      k_dbg_safe2<<<blocks_for(L.n, 256, 65536), 256, 0, s>>>(L.safe_root, L.pos, d_poff, L.njobs,
                                                               L.n, minid, out);
      PCC_HIP(hipMemcpyAsync(host_dst, out + L.p_off[q], n_job * sizeof(int32_t),
                             hipMemcpyDeviceToHost, s));
      PCC_HIP(hipStreamSynchronize(s));
      return PCC_OK;
    }
    if (what == PCC_DBG_EDITABLE) {
      const size_t ne = L.ne ? L.ne : 1;
      int32_t *jb = scratch.get<int32_t>(ne);
      uint32_t *id = scratch.get<uint32_t>(ne);
      if (L.ne)
        k_dbg_e<<<blocks_for(L.ne, 256, 65536), 256, 0, s>>>(L.e_list, L.ne, L.pos, d_poff, L.njobs,
                                                            jb, id);
      std::vector<int32_t> hj(L.ne);
      std::vector<uint32_t> hid(L.ne);
      if (L.ne) {
        PCC_HIP(hipMemcpyAsync(hj.data(), jb, L.ne * 4, hipMemcpyDeviceToHost, s));
        PCC_HIP(hipMemcpyAsync(hid.data(), id, L.ne * 4, hipMemcpyDeviceToHost, s));
      }
      PCC_HIP(hipStreamSynchronize(s));
      std::vector<uint32_t> sel;
      for (size_t e = 0; e < L.ne; ++e)
        if (hj[e] == q) sel.push_back(hid[e]);
      *count = (int64_t)sel.size();
      if (host_dst && cap >= *count) std::memcpy(host_dst, sel.data(), sel.size() * 4);
      return PCC_OK;
    }
    if (what == PCC_DBG_ACTIVE_I || what == PCC_DBG_ACTIVE_J || what == PCC_DBG_ACTIVE_TYPE ||
        what == PCC_DBG_ACTIVE_THR) {
      const size_t na = L.na ? L.na : 1;
      int32_t *jb = scratch.get<int32_t>(na);
      uint32_t *lo = scratch.get<uint32_t>(na), *hi = scratch.get<uint32_t>(na);
      uint8_t *t = scratch.get<uint8_t>(na), *tk = scratch.get<uint8_t>(na);
      if (L.na)
        k_dbg_pairs<<<blocks_for(L.na, 256, 65536), 256, 0, s>>>(L.a_i, L.a_j, L.a_t, L.a_k, L.na,
                                                                 L.pos, d_poff, L.njobs, jb, lo,
                                                                 hi, t, tk);
      std::vector<int32_t> hj(L.na);
      std::vector<uint32_t> hl(L.na), hh(L.na);
      std::vector<uint8_t> ht(L.na), hk(L.na);
      if (L.na) {
        PCC_HIP(hipMemcpyAsync(hj.data(), jb, L.na * 4, hipMemcpyDeviceToHost, s));
        PCC_HIP(hipMemcpyAsync(hl.data(), lo, L.na * 4, hipMemcpyDeviceToHost, s));
        PCC_HIP(hipMemcpyAsync(hh.data(), hi, L.na * 4, hipMemcpyDeviceToHost, s));
        PCC_HIP(hipMemcpyAsync(ht.data(), t, L.na, hipMemcpyDeviceToHost, s));
        PCC_HIP(hipMemcpyAsync(hk.data(), tk, L.na, hipMemcpyDeviceToHost, s));
      }
      PCC_HIP(hipStreamSynchronize(s));
      int64_t c = 0;
      for (size_t p = 0; p < L.na; ++p) c += hj[p] == q;
      *count = c;
      if (!host_dst || cap < c) return PCC_OK;
      int64_t w = 0;
      for (size_t p = 0; p < L.na; ++p) {
        if (hj[p] != q) continue;
        if (what == PCC_DBG_ACTIVE_I) ((uint32_t *)host_dst)[w] = hl[p];
        if (what == PCC_DBG_ACTIVE_J) ((uint32_t *)host_dst)[w] = hh[p];
        if (what == PCC_DBG_ACTIVE_TYPE) ((uint8_t *)host_dst)[w] = ht[p];
        if (what == PCC_DBG_ACTIVE_THR) ((uint8_t *)host_dst)[w] = hk[p];
        ++w;
      }
      return PCC_OK;
    }
    return fail(PCC_E_INVALID_ARG, "unknown debug item");
  });
}
