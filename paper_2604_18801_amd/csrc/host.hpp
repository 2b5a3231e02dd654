// Host-side pieces of the library: context, batch pipeline, edit-stream
// codec (canonical Huffman + ZSTD through the runtime libzstd).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pcc.h"
#include "kernels.hpp"

namespace pcc {

// Retained device data of the last call (test hook pcc_debug_fetch).
struct LastCall {
  bool valid = false;
  int njobs = 0;
  std::vector<int64_t> p_off;      // [njobs+1] particles per job (global space)
  std::vector<int> job_index;      // caller job index of each included job
  size_t n = 0, na = 0, ne = 0;
  const uint32_t *a_i = nullptr, *a_j = nullptr;
  const uint8_t *a_t = nullptr;
  const uint8_t *a_k = nullptr;    // threshold index per pair (multi-threshold calls)
  const uint32_t *safe_root = nullptr;
  const float4 *pos = nullptr;
  const uint32_t *e_list = nullptr;
  // cell list of the call (all jobs): cell starts [n_cells + 1] and the 13
  // forward neighbour cells of each cell (-1: none)
  const uint32_t *cell_start = nullptr;
  const uint2 *nrange = nullptr;  // [cells][kNbrSlots]
  const uint32_t *n_cells = nullptr;
};

// Adam bias corrections (1 - beta1^t, 1 - beta2^t) for t = 0 .. len - 1,
// computed on the host with the C library's pow and kept on the device.
struct BcTable {
  double beta1, beta2;
  int64_t len;
  double2 *dev;
};

// Optional HIP-event brackets around kernel launches.
struct KernelTimer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, int>> marks;  // (kernel id, first event index)
  size_t used = 0;
  double acc_ms[PCC_NKERNELS] = {};  // times of graph replays already read
  int64_t acc_n[PCC_NKERNELS] = {};
  void begin_call() {
    marks.clear();
    used = 0;
    for (int k = 0; k < PCC_NKERNELS; ++k) acc_ms[k] = 0.0, acc_n[k] = 0;
  }
  void reserve(size_t n);  // at least n unused events in the pool
  void record(hipEvent_t e, hipStream_t s);
  int start(int id, hipStream_t s);
  void stop(int at, hipStream_t s);
  // an event pair around a graph replay (reused by the next replay, after
  // add_split has read it): the replay's time counts as k launches of id
  int bracket_begin(hipStream_t s);
  void bracket_end(int at, hipStream_t s);
  void add_split(int id, int at, int k);
  // per kernel id: the accumulators plus the marks of direct launches
  void collect(double *ms, int64_t *count);
  ~KernelTimer();
};

class PgdEngine;

// The instantiated PGD graph of the last call, kept for the next call whose
// launches are identical (same buffers and sizes: the same job shapes on a
// workspace laid out the same way), which then skips capture and
// instantiation.
struct PgdGraphCache {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  PgdBufs bufs{};
  const PgdGroups *groups = nullptr;
  int steps = 0;
  void clear() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    groups = nullptr;
    steps = 0;
  }
};

struct Context {
  int device = 0;
  // served form: the shared PGD loop this context's calls join (none for a
  // plain context)
  PgdEngine *engine = nullptr;
  KernelTimer kt;
  int graph_iters = 8;
  bool force_exact_pairs = false;  // always count the kept pairs before writing them
  // scheduling knobs (results do not depend on them; pcc_autotune picks them)
  int cell_pct = 100;    // cell side as a percentage of r_v (>= 100)
  int dense_cell = 32;   // cells with at least this many particles take the dense pair path
  std::vector<BcTable> bc;
  hipStream_t own = nullptr;
  PgdGraphCache pgd_graph;
  Arena arena;
  LastCall last;
  hipEvent_t ev[12] = {};
  void *pinned = nullptr;        // small pinned staging buffer
  size_t pinned_bytes = 0;
  void *pinned_big = nullptr;    // staging for stream bytes
  size_t pinned_big_bytes = 0;
};

// longest bias-correction table a job may read: 2^24 entries (256 MiB)
constexpr int64_t kMaxBcTable = (int64_t)1 << 24;
// entries of the table a job with these betas and cap reads
int64_t bc_length(double beta1, double beta2, int64_t max_iters);
const double2 *bc_table(Context &C, double beta1, double beta2, int64_t len);

// message returned by pcc_last_error on the calling thread
void set_last_error(const std::string &m);

// tune.cpp: times the jobs under candidate scheduling knobs and leaves the
// fastest on the context
void autotune(Context &C, const pcc_job *jobs, int njobs, hipStream_t s, int32_t flags,
              pcc_tune_report &rep);

// multi: the jobs are one snapshot at several linking lengths, corrected
// together into job 0's particles (job 0's stream; every job's labels)
// scratch: labels only, every device buffer of the call from this fixed
// arena (no device or pinned allocation, no kernel timing, the context's
// arena and retained debug data untouched)
// footprint: run only through pair pass 1 and the slot counts, and store a
// bound of the workspace bytes the whole call takes
pcc_status run_batch(Context &C, const pcc_job *jobs, int njobs, pcc_job_result *res,
                     hipStream_t s, bool labels_only, bool multi = false,
                     Arena *scratch = nullptr, size_t *footprint = nullptr);
// stage events of a context (created once, with the context)
void create_events(Context &C);

// engine.cpp: the shared PGD loop of the served form.  engine_run adds the
// group gb (past its first step and renumbering, `active` jobs not done) to
// the loop and returns when every job of it is done.
PgdEngine *engine_create(int device, int graph_iters);
void engine_destroy(PgdEngine *e);
void engine_run(PgdEngine *e, const PgdBufs &gb, int32_t active);
// scratch.hip: finds the device address of the static scratch of the
// allocation-free calls on `device` (the current device), once per device
void scratch_init(int device);
// static-scratch bytes the last allocation-free call used
int64_t noalloc_high_water();

// codec.cpp
struct HuffTable {
  std::vector<uint32_t> syms;   // symbols with a code, in (length, symbol) order
  std::vector<uint8_t> lens;
  std::vector<uint32_t> table;  // [65536] reversed code | length << 24
};
void huffman_build(const uint32_t *hist, int alphabet, HuffTable &out);
bool zstd_available();
// returns false when ZSTD is unavailable or fails; dst gets the frame
bool zstd_compress(const uint8_t *src, size_t len, std::vector<uint8_t> &dst, int level);
bool zstd_decompress(const uint8_t *src, size_t len, uint8_t *dst, size_t raw_len);
size_t stream_bound(int64_t n, int m_bits);
// header + payload assembly
// symbols per chunk of the Huffman bitstream's chunk index
constexpr uint32_t kHuffChunk = 4096;
void assemble_stream(int64_t n, int m_bits, int64_t nflagged, double qstep, double qoffset,
                     const uint8_t *flags, size_t nflag_bytes, const HuffTable *ht,
                     const uint32_t *words, uint64_t nbits, const uint64_t *chunk_bits,
                     size_t nchunks, std::vector<uint8_t> &out, size_t *payload_raw);
// a stream's flags (first flag_bytes bytes of payload, bit k of byte k/8)
// and its symbols (planes x, y, z over the flagged particles in increasing
// index; m = 32 codes are a low then a high 16-bit symbol)
struct ParsedStream {
  int64_t n = 0;
  uint64_t nflagged = 0;
  int per = 1;
  double step = 0.0, offset = 0.0;
  size_t flag_bytes = 0;
  std::vector<uint8_t> payload;
  // symbols: decoded on the host, or (Huffman left to the device) empty
  std::vector<uint32_t> sym;
  // Huffman section: the symbols in canonical order (length, then value)
  // with their code lengths, the bitstream and its chunk index, both at
  // byte offsets of payload
  bool huff = false;
  std::vector<uint32_t> canon_sym;
  std::vector<uint8_t> canon_len;
  uint64_t nbits = 0;
  uint32_t chunk = 0;
  size_t nchunks = 0, index_at = 0, bits_at = 0;
};
// huffman_on_host: decode the Huffman bitstream here (else only its tables
// and chunk index are parsed, for the device decoder)
pcc_status parse_stream(const uint8_t *stream, size_t len, int64_t n, ParsedStream &out,
                        std::string &err, bool huffman_on_host);
// applies a parsed stream to a device reconstruction (decode.hip), the
// Huffman bitstream decoded on the device; false when it is corrupt
bool apply_edits_device(const ParsedStream &ps, const float *const rin[3], float *const rout[3],
                        Arena &ar, hipStream_t s);
pcc_status decode_stream(const uint8_t *stream, size_t len, int64_t n, const float *rx,
                         const float *ry, const float *rz, float *ox, float *oy, float *oz,
                         std::string &err);

}  // namespace pcc

// the opaque handle of the C ABI
struct pcc_context {
  pcc::Context c;
};
