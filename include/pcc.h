/*
 * pcc.h -- C ABI of the MI355X (gfx950) library for cluster-preserving
 * correction of lossy-compressed particle data.
 *
 * The method is that of "Preserving Clusters in Error-Bounded Lossy
 * Compression of Scientific Particle Data" (Ren, Di, Heitmann, Cappello,
 * Guo).  Its problem statement (Alg. 1: original positions P, base-compressed
 * positions P^(0), error bound xi, linking length b, bit depth m, learning
 * rate alpha, iteration cap T_max, loss tolerance eps_L and mode in; the
 * compressed edit stream out) is the shape of pcc_correct.  The library adds
 * the friends-of-friends labels of P (Sec. 2.4), a batched entry point for
 * many independent snapshots, and a decoder (Sec. 3.3, "Reconstruction of
 * the edited data").
 *
 * Conventions
 *   - Every call returns a pcc_status; negative values are errors, the
 *     message of the last error of the calling thread is pcc_last_error().
 *   - Positions are structure-of-arrays float32 (x, y, z), n entries each.
 *     pcc_particles.memspace says whether the pointers are host memory or
 *     device memory of the context's GPU.  The library only reads them and
 *     does not keep them after the call returns.
 *   - Outputs are caller-allocated; the library allocates none.  Labels are
 *     written to memory of the same memspace as the original particles.
 *   - Work is queued on the HIP stream passed as `hip_stream` (NULL = the
 *     default stream); a call returns when its results are complete.
 *   - A context is bound to one device and is not thread-safe: calls that
 *     share a context must not overlap.
 */
#ifndef PCC_H
#define PCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PCC_VERSION 1

typedef int32_t pcc_status;
enum {
  PCC_OK = 0,
  PCC_NOT_CONVERGED = 1,      /* warning: T_max reached with violations left;
                                 the outputs are valid and inside the box */
  PCC_PENDING = 2,            /* server: the job is queued or running */
  PCC_E_INVALID_ARG = -1,     /* b <= 0, xi < 0, NaN/Inf input, m not in
                                 {8,16,32}, n < 0, periodic side < 3 (b +
                                 2 sqrt(3) xi), n >= 2^31, NULL pointers */
  PCC_E_OUT_OF_MEMORY = -2,
  PCC_E_DEVICE = -3,          /* a HIP runtime call failed */
  PCC_E_BUFFER_TOO_SMALL = -4,/* stream_cap too small; *stream_len = need */
  PCC_E_INPUT_BOUND = -5,     /* some |x_hat - x| > xi (Sec. 3.1 assumes
                                 the base compressor honours the bound) */
  PCC_E_UNSUPPORTED = -6,
  PCC_E_CANCELLED = -7
};

/* constraint-selection modes, Sec. 3.2 */
enum { PCC_MODE_VP = 0, PCC_MODE_SC = 1, PCC_MODE_HF = 2 };
/* optimiser: Adam (Sec. 4.2) or the plain step printed in Alg. 1 */
enum { PCC_OPT_ADAM = 0, PCC_OPT_SGD = 1 };
/* safety margins, Sec. 3.3: SAFE also covers float32 rounding of the
   decoded coordinates; PAPER uses xi(1 - 2^-m) and 2 sqrt(3) eps_q */
enum { PCC_MARGIN_SAFE = 0, PCC_MARGIN_PAPER = 1 };
enum { PCC_MEM_HOST = 0, PCC_MEM_DEVICE = 1 };

typedef struct pcc_context pcc_context;

/* Borrowed view of n particles, float32 structure of arrays. */
typedef struct {
  const float *x, *y, *z;
  int64_t n;
  int32_t memspace;  /* PCC_MEM_HOST or PCC_MEM_DEVICE */
  int32_t reserved;
} pcc_particles;

/* Alg. 1 inputs; pcc_params_init fills the defaults. */
typedef struct {
  double b;              /* linking length, > 0 */
  double xi;             /* absolute pointwise error bound, >= 0 */
  int32_t mode;          /* PCC_MODE_*, default HF */
  int32_t m_bits;        /* bit depth of quantised edits: 8, 16 (default), 32 */
  int32_t optimizer;     /* PCC_OPT_*, default Adam */
  int32_t margin_policy; /* PCC_MARGIN_*, default SAFE */
  double lr;             /* alpha, default 1e-3 */
  double beta1, beta2;   /* Adam, default 0.9, 0.999 */
  double adam_eps;       /* Adam epsilon, default 1e-8 */
  int64_t max_iters;     /* T_max; <= 0 selects the safety cap 100000; at most
                            2^31 (larger: PCC_E_INVALID_ARG) */
  double loss_tol;       /* eps_L; 0 (default) stops when no selected pair is
                            violated, > 0 stops when the tightened loss of
                            Eq. 3 is <= loss_tol.  The loss is summed in
                            float64 in a fixed order that differs from a
                            sequential sum over the pairs (relative
                            difference ~1e-15) */
  double box[3];         /* periodic side per axis; 0 = open axis (default) */
} pcc_params;

/* Caller-allocated outputs of one correction. */
typedef struct {
  int32_t *labels;       /* [n] FoF labels of the originals (smallest member
                            index), memspace of the originals; may be NULL */
  uint8_t *stream;       /* host buffer for the edit stream; may be NULL
                            together with stream_cap = 0 */
  size_t stream_cap;
  size_t *stream_len;    /* host; set to the stream size (or the size needed) */
  double *debug_xyz;     /* host [3][n] planar float64 coordinates before
                            quantisation (the reconstruction for particles
                            that were not edited); may be NULL */
  /* Per-evaluation trace of the loop of Alg. 1 (the loss-against-iteration
     curve of Sec. 4): entry t holds the tightened loss of Eq. 3 (float64)
     and the number of violated selected constraints at iterate t, for
     t = 0 .. min(iters, trace_cap - 1).  Host buffers of trace_cap entries;
     either may be NULL (then trace_cap is ignored for it). */
  double *loss_trace;
  int64_t *viol_trace;
  int64_t trace_cap;
} pcc_outputs;

#define PCC_NSTAGES 10
/* stage timings, milliseconds of device time measured with HIP events:
   0 input scan, 1 cell build, 2 pair pass (classify + components),
   3 labels, 4 constraint selection, 5 editable set and CSR, 6 PGD,
   7 device encoding, 8 host lossless stage, 9 total wall time */
#define PCC_NKERNELS 8
/* device time of the main kernels, summed over their launches, filled only
   when kernel timing is on (pcc_context_set): 0 pair classify/hook pass,
   1 pair count pass, 2 pair write pass, 3 PGD step, 4 PGD finalize,
   5 cell-key sort, 6 pair and incidence sorts, 7 spanning-forest rounds */
typedef struct {
  int64_t n_pairs;       /* pairs with d <= b + 2 sqrt(3) xi */
  int64_t n_safe, n_pb, n_pc;
  int64_t n_active, n_editable, n_flagged;
  int64_t iters;         /* gradient steps taken */
  double loss0, loss_final;
  int64_t viol0, viol_final;
  int64_t bytes_flags, bytes_codes, bytes_stream;
  double t_stage_ms[PCC_NSTAGES];
  double kernel_ms[PCC_NKERNELS];
  int64_t kernel_launches[PCC_NKERNELS];
  /* work of the PGD steps, summed over all steps: rows (editable particles)
     and row incidences whose constraints were evaluated; a row is skipped
     in a step when it is an exact fixed point of that step */
  int64_t pgd_rows_evaluated, pgd_incidences_evaluated;
} pcc_stats;

typedef struct {
  pcc_particles orig;
  pcc_particles recon;
  pcc_params params;
  pcc_outputs out;
} pcc_job;

typedef struct {
  pcc_status status;
  int32_t reserved;
  pcc_stats stats;
  /* served jobs only (zero otherwise): milliseconds since the server was
     created at which the job was submitted, its batch started and the job
     finished; the number of jobs in its batch and the worker that ran it */
  double t_submit_ms, t_start_ms, t_finish_ms;
  int32_t batch_jobs, worker;
} pcc_job_result;

int pcc_version(void);
const char *pcc_status_string(pcc_status s);
/* Thread-local message of the last error on this thread ("" if none). */
const char *pcc_last_error(void);

pcc_status pcc_context_create(int device, pcc_context **out);
pcc_status pcc_context_destroy(pcc_context *ctx);

/*
 * Context options.
 *   PCC_CTX_KERNEL_TIMING  0/1: bracket the main kernels with HIP events and
 *                          report their device time in pcc_stats.kernel_ms.
 *                          A captured PGD graph is timed as a whole and its
 *                          time split evenly over its steps: kernel_ms of
 *                          the PGD step then includes the finalize launch of
 *                          those steps, whose own count and time cover only
 *                          the first (direct) step.  Default 0.
 *   PCC_CTX_GRAPH_ITERS    PGD iterations per captured graph launch (1..64,
 *                          default 8); one small readback follows each launch.
 *   PCC_CTX_EXACT_PAIRS    0/1: always count the pairs a mode keeps in a pass
 *                          of its own before writing them (the path taken
 *                          anyway when the slots sized by the pair classes
 *                          would not fit in half the free device memory).
 *                          Results are the same either way.  Default 0.
 */
enum {
  PCC_CTX_KERNEL_TIMING = 1,
  PCC_CTX_GRAPH_ITERS = 2,
  PCC_CTX_EXACT_PAIRS = 3,
  PCC_CTX_CELL_PCT = 4,
  PCC_CTX_DENSE_CELL = 5,
  PCC_CTX_WORKSPACE_HIGH_WATER = 6
};
/*
 * Scheduling knobs (no result depends on them; pcc_autotune sets them):
 *   PCC_CTX_CELL_PCT       side of the cell-list cells as a percentage of
 *                          r_v = b + 2 sqrt(3) xi, 100 .. 400 (default 100).
 *                          Cells are never smaller than r_v, so the 13
 *                          forward neighbour cells hold every partner; a
 *                          periodic axis keeps at least three cells.
 *   PCC_CTX_DENSE_CELL     cells with at least this many particles are
 *                          searched by whole waves (64 home particles per
 *                          wave, partners staged through LDS), the others by
 *                          one thread per particle; 1 .. 4096 (default 32).
 *   PCC_CTX_WORKSPACE_HIGH_WATER  (get only) device workspace bytes the last
 *                          call on the context used at most.
 */
pcc_status pcc_context_set(pcc_context *ctx, int32_t key, int64_t value);
/* Reads a context option (any key above) into *value. */
pcc_status pcc_context_get(pcc_context *ctx, int32_t key, int64_t *value);

/*
 * Autotuner: corrects the jobs (the same list pcc_correct_batch takes;
 * their outputs are not written) under candidate scheduling knobs on this
 * context's device and leaves the fastest on the context.  First the cell
 * side (PCC_CTX_CELL_PCT 100, 125, 150, 200) and the dense-cell threshold
 * (16, 32, 64, 128), each pair scored by the device time of the stages they
 * act on (cell build, pair passes, labels, selection, CSR); then, unless
 * flags has PCC_TUNE_NO_GRAPH, the PGD graph length (PCC_CTX_GRAPH_ITERS 4,
 * 8, 16, 32) scored by the wall time of the call.  Every trial is recorded
 * in rep (may be NULL).
 * Work is queued on hip_stream; the call returns when it is done.  The jobs'
 * results do not depend on the knobs, only their speed.
 */
#define PCC_TUNE_MAX_TRIALS 32
enum { PCC_TUNE_NO_GRAPH = 1 };
typedef struct {
  int32_t cell_pct, dense_cell, graph_iters;  /* chosen (now set on the context) */
  int32_t n_trials;
  int32_t trial_kind[PCC_TUNE_MAX_TRIALS];    /* 0 stages before PGD, 1 whole call */
  int32_t trial_cell_pct[PCC_TUNE_MAX_TRIALS];
  int32_t trial_dense_cell[PCC_TUNE_MAX_TRIALS];
  int32_t trial_graph_iters[PCC_TUNE_MAX_TRIALS];
  double trial_ms[PCC_TUNE_MAX_TRIALS];       /* its score in ms */
} pcc_tune_report;
pcc_status pcc_autotune(pcc_context *ctx, const pcc_job *jobs, int32_t njobs, int32_t flags,
                        pcc_tune_report *rep, void *hip_stream);

void pcc_params_init(pcc_params *p);

/* Upper bound of the edit stream size for n particles. */
size_t pcc_stream_bound(int64_t n, const pcc_params *p);

/*
 * The correction pass of Alg. 1 on one snapshot: cell build, pair search and
 * classification (Sec. 3.1), FoF and safe components (Sec. 2.4, 3.2),
 * constraint selection (Sec. 3.2), PGD with Adam and box projection
 * (Alg. 1, Eq. 2-3), edit encoding (flags, m-bit edits, Huffman + ZSTD).
 * orig and recon must have the same n and memspace.  stats may be NULL.
 * Returns PCC_OK, PCC_NOT_CONVERGED or an error.
 */
pcc_status pcc_correct(pcc_context *ctx, const pcc_particles *orig,
                       const pcc_particles *recon, const pcc_params *params,
                       pcc_outputs *out, pcc_stats *stats, void *hip_stream);

/*
 * One snapshot corrected for several linking lengths at once (the extension
 * the conclusion names, Sec. 5 under Limitations: the constraints of every
 * threshold are selected as in pcc_correct, with that threshold's
 * b -+ delta_t, and the loss of Eq. 3 sums over their union; a pair selected
 * by two thresholds counts twice).
 * b_list[0 .. nb) (1 <= nb <= PCC_MAX_THRESHOLDS, each finite and > 0)
 * replaces params->b; every other parameter applies to all thresholds.
 * out->labels, if not NULL, receives the FoF labels of the originals at every
 * linking length, [nb][n] row-major, in the memspace of orig; the stream,
 * debug_xyz and stats are those of the one corrected snapshot (the pair
 * counts in stats are those at b_list[0]).  The PGD row of a particle sums
 * its constraints in increasing partner index, then threshold index.
 * Returns as pcc_correct.
 */
#define PCC_MAX_THRESHOLDS 8
pcc_status pcc_correct_multi(pcc_context *ctx, const pcc_particles *orig,
                             const pcc_particles *recon, const pcc_params *params,
                             const double *b_list, int32_t nb, pcc_outputs *out,
                             pcc_stats *stats, void *hip_stream);

/*
 * Many independent snapshots in one pass: every stage is one launch over all
 * jobs, the PGD iterations of all jobs run together and a job that has
 * converged is masked out.  Each job's results equal those of pcc_correct on
 * that job alone.  results[k].status holds each job's status; the return
 * value is PCC_OK unless a job failed (then the first job error).
 * 0 <= njobs <= PCC_MAX_BATCH_JOBS (else PCC_E_INVALID_ARG, nothing run).
 */
#define PCC_MAX_BATCH_JOBS 65536
pcc_status pcc_correct_batch(pcc_context *ctx, const pcc_job *jobs, int32_t njobs,
                             pcc_job_result *results, void *hip_stream);

/*
 * Decode an edit stream and apply it to the reconstruction (Sec. 3.3):
 * out = float32(x_hat + edit) for flagged particles, x_hat bit-exactly for
 * the others.  recon and out are host arrays of n entries each.
 */
pcc_status pcc_decode(const uint8_t *stream, size_t len, const pcc_particles *recon,
                      float *out_x, float *out_y, float *out_z);

/*
 * The same decoding with device arrays (recon and out on the context's GPU):
 * the host undoes ZSTD and reads the stream's tables (flag mask, canonical
 * Huffman code, chunk index); the Huffman bitstream is decoded on the GPU,
 * one thread per chunk of 4096 symbols starting at the bit the stream's
 * chunk index gives, and a kernel applies the edits; the output equals
 * pcc_decode's bit for bit.  A bitstream whose codes do not end exactly at
 * the next chunk start, or code lengths that no prefix code has, give
 * PCC_E_INVALID_ARG with the output untouched.  Work is queued on
 * hip_stream and the call returns when it is done.  Invalidates the
 * context's retained debug data.
 */
pcc_status pcc_decode_device(pcc_context *ctx, const uint8_t *stream, size_t len,
                             const pcc_particles *recon, float *out_x, float *out_y,
                             float *out_z, void *hip_stream);

/*
 * Device workspace a pcc_correct of these inputs would take at most, for
 * admission by footprint (the served form uses it): the call's stages run
 * up to the first pair pass (cells, pair classes and their per-particle
 * counts, Sec. 3.1-3.3) and the rest is bounded from those counts (the
 * slots for every vulnerable pair the mode may keep, the spanning-forest
 * candidates, the CSR, the PGD state and the encoder); the bound is at
 * least the workspace high water of the full call.  Inputs as for
 * pcc_correct (device or host); the work is queued on hip_stream and the
 * call returns when it is done.  Status as for pcc_correct's input checks.
 */
pcc_status pcc_workspace_query(pcc_context *ctx, const pcc_particles *orig,
                               const pcc_particles *recon, const pcc_params *params,
                               size_t *bytes, void *hip_stream);

/*
 * Friends-of-friends labels (Sec. 2.4) of a point set at linking length b:
 * labels[k] is the smallest index in k's cluster.  box as in pcc_params.
 * labels has the memspace of pts.
 */
pcc_status pcc_fof_labels(pcc_context *ctx, const pcc_particles *pts, double b,
                          const double box[3], int32_t *labels, void *hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * labels as pcc_fof_labels, bit for bit, computed by the same kernels, with
 * every device buffer taken from a static device array of 128 MiB that the
 * library holds on each GPU it runs on until the process ends.  The call
 * makes no hipMalloc / hipFree / hipHostMalloc and creates no HIP object;
 * the caller passes the points and the labels buffer (memspace of pts; host
 * inputs are staged through the static array).  n above
 * pcc_fof_labels_noalloc_max_n() (520192) returns PCC_E_INVALID_ARG before
 * any device work.  The array keeps the last call's contents; the call
 * initialises everything it reads.  Calls on one GPU share the one array:
 * within a process they are serialised by a lock (each returns only when
 * its work on hip_stream has finished); calls that overlap on one GPU
 * without it (e.g. work still queued by a caller that ignored an error)
 * would race.  The context supplies the device, its scheduling knobs and
 * its stage events; its workspace and retained debug data are not touched.
 */
pcc_status pcc_fof_labels_noalloc(pcc_context *ctx, const pcc_particles *pts, double b,
                                  const double box[3], int32_t *labels, void *hip_stream);
int64_t pcc_fof_labels_noalloc_max_n(void);

/*
 * Test hook: copy an intermediate result of job `job` of the last
 * pcc_correct / pcc_correct_batch call on this context into host memory.
 * Pair lists use particle indices of the job with i < j, unsorted.
 *   PCC_DBG_ACTIVE_I / _J   uint32 [n_active]  active pairs
 *   PCC_DBG_ACTIVE_TYPE     uint8  [n_active]  2 = potentially broken,
 *                                              3 = potentially created
 *   PCC_DBG_SAFE_LABELS     int32  [n]         safe-component labels
 *   PCC_DBG_EDITABLE        uint32 [n_editable] editable particles, unsorted
 *   PCC_DBG_ACTIVE_THR      uint8  [n_active]  linking-length index of each
 *                                              active pair (0 outside
 *                                              pcc_correct_multi)
 *   PCC_DBG_CELL_START      uint32 [cells + 1] first sorted particle of each
 *                                              non-empty cell of the call (all
 *                                              jobs), then the particle count
 *   PCC_DBG_NEIGHBORS       uint32 [18 cells]  the 13 forward neighbour cells
 *                                              of each cell as 9 ranges
 *                                              (first, end) of sorted
 *                                              particles, first == end
 *                                              where empty
 * *count receives the element count; nothing is copied if cap < count.
 */
enum {
  PCC_DBG_ACTIVE_I = 1,
  PCC_DBG_ACTIVE_J = 2,
  PCC_DBG_ACTIVE_TYPE = 3,
  PCC_DBG_SAFE_LABELS = 4,
  PCC_DBG_EDITABLE = 5,
  PCC_DBG_ACTIVE_THR = 6,
  PCC_DBG_CELL_START = 7,
  PCC_DBG_NEIGHBORS = 8
};
pcc_status pcc_debug_fetch(pcc_context *ctx, int32_t job, int32_t what, void *host_dst,
                           int64_t cap, int64_t *count);

/*
 * Test hook for failure handling (process-wide, no device call):
 *   PCC_DEBUG_ALLOC_FAIL_AFTER  value >= 0: after `value` more successful
 *                               workspace allocations, the next one fails as
 *                               if the device were out of memory (the call
 *                               then returns PCC_E_OUT_OF_MEMORY, or a
 *                               server retries the jobs of that batch one
 *                               by one); the hook then switches itself off.
 *                               value -1 switches it off.
 * pcc_debug_get reads the current value (the allocations left before the
 * failure, or a negative number when off).
 *   PCC_DEBUG_NOALLOC_HIGH_WATER  (get only) bytes of the static array the
 *                               last pcc_fof_labels_noalloc call used.
 */
enum { PCC_DEBUG_ALLOC_FAIL_AFTER = 1, PCC_DEBUG_NOALLOC_HIGH_WATER = 2 };
pcc_status pcc_debug_set(int32_t key, int64_t value);
pcc_status pcc_debug_get(int32_t key, int64_t *value);

/*
 * Served form: a job queue in front of the batched pass, with
 * iteration-level continuous batching.  Slot threads (n_streams of them,
 * each with its own HIP stream and workspace on the context's device) take
 * the queued jobs in arrival order, as many together as max_inflight and
 * their share of hbm_budget allow, and run every stage up to the first PGD
 * step on their own streams.  The PGD iterations of every prepared call then
 * run in one shared loop (one stream, a captured graph of K steps over all
 * resident calls): a call joins it between two replays and leaves it, to be
 * encoded on its slot's stream, at the end of the replay in which its last
 * job converged, so jobs that arrive while others iterate overlap with them
 * and no job waits for a slower one.  Each job's results equal those of
 * pcc_correct on that job alone.  When a batch runs out of device memory its jobs are run
 * again one at a time, and a job that runs out of memory alone gets one
 * more try after its worker's workspace is released.  Job buffers are borrowed until the job has finished;
 * device inputs must be ready (their producing stream synchronised) when
 * the job is submitted.  The server's calls are thread-safe; the context is
 * used only to pick the device and its options, and stays the caller's.
 */
typedef struct pcc_server pcc_server;
typedef struct {
  size_t hbm_budget;     /* device bytes the workers may use together; 0 = 80%
                            of the free memory at creation */
  int32_t max_inflight;  /* jobs per batch at most; 0 = 256 */
  int32_t n_streams;     /* calls in flight at once (slots), 0 .. 32; 0 = 16 */
} pcc_server_config;

pcc_status pcc_server_create(pcc_context *ctx, const pcc_server_config *cfg,
                             pcc_server **out);
/* Queue a job; never blocks.  *ticket identifies it in the calls below. */
pcc_status pcc_server_submit(pcc_server *srv, const pcc_job *job, uint64_t *ticket);
/* PCC_PENDING while the job is queued or running, else the job's status
   (and *result filled; result may be NULL). */
pcc_status pcc_server_poll(pcc_server *srv, uint64_t ticket, pcc_job_result *result);
/* Like poll, but blocks up to timeout_ms (negative: no limit). */
pcc_status pcc_server_wait(pcc_server *srv, uint64_t ticket, int64_t timeout_ms,
                           pcc_job_result *result);
/* Remove a job that has not started: PCC_OK, and the job's status becomes
   PCC_E_CANCELLED.  A job that has started runs to completion
   (PCC_E_INVALID_ARG, as for an unknown ticket). */
pcc_status pcc_server_cancel(pcc_server *srv, uint64_t ticket);
/* Block until every submitted job has finished. */
pcc_status pcc_server_drain(pcc_server *srv);
/* Drain, stop the workers and free the server. */
pcc_status pcc_server_destroy(pcc_server *srv);

#ifdef __cplusplus
}
#endif
#endif
