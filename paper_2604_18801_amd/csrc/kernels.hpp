// Host launchers of the correction kernels (one translation unit per stage).
#pragma once

#include "pcc_internal.hpp"

namespace pcc {

// Input scan partial of one tile (a range of one job's particles).
struct ScanPart {
  float mn[3], mx[3];
  float maxabs;
  uint32_t bad_bound;   // |x_hat - x| > xi
  uint32_t bad_value;   // NaN or Inf
  uint32_t job;
};
struct Tile {
  int64_t start, end;
  int32_t job, pad;
};
// three float32 coordinate arrays (x, y, z) of the global index space
struct Soa3 {
  const float *a[3];
};

// cells.hip
void launch_scan_inputs(const Tile *tiles, int ntiles, Soa3 orig3,
                        Soa3 rec3, const double *xi_job, ScanPart *parts,
                        hipStream_t s);
void launch_cell_keys(const JobDev *jobs, const int64_t *p_off, int njobs,
                      Soa3 orig3, size_t n, uint32_t *keys, uint32_t *vals,
                      hipStream_t s);
void launch_gather(const uint32_t *perm, const int64_t *p_off, int njobs,
                   Soa3 orig3, Soa3 rec3, size_t n,
                   float4 *pos, float4 *rec, uint32_t *inv_perm, hipStream_t s);
// unique cells of the sorted keys; returns device counter of unique cells
void build_cells(const uint32_t *keys, size_t n, uint32_t *cell_of, uint32_t *cell_start,
                 uint32_t *cell_key, uint32_t *n_cells, Arena &ar, hipStream_t s);
// Forward neighbours of each cell as kNbrSlots particle ranges [x, y) of the
// sorted order (empty when x == y); key_space: one more than the largest
// cell key of any job
constexpr int kNbrSlots = 9;
void launch_neighbors(const JobDev *jobs, const uint32_t *cell_base, int njobs,
                      const uint32_t *cell_key, const uint32_t *n_cells, const uint32_t *cell_start,
                      size_t max_cells, uint64_t key_space, uint2 *nrange, uint8_t *edge,
                      Arena &ar, hipStream_t s);

// pairs.hip
struct PairBufs {
  const JobDev *jobs;
  const int64_t *p_off;
  int njobs;
  size_t n;
  const float4 *pos, *rec;
  const uint32_t *cell_of, *cell_start;
  const uint2 *nrange;                   // [cell][kNbrSlots] forward neighbour particle ranges
  const uint8_t *cell_edge;              // periodic faces of each cell (image shifts)
  uint32_t *safe_par, *fof_par;          // union-find parents (sorted space)
  uint32_t *cnt_pb, *cnt_pc;             // pass 1: pb and pc pairs of each home particle
  uint32_t *cnt_a, *cnt_f;               // pass 2: active and forest pairs (exact path);
                                         // pass 3: filled active slots (slotted path)
  const uint32_t *cap_f;                 // slotted path: forest slots of each home particle
  int slotted;                           // pass 3 writes into slots sized by pass 1
  unsigned long long *job_counts;        // [njobs][count_slots][16]: safe, pb, pc partial sums
  int count_slots;                       // power of two
  const uint64_t *off_a, *off_f;         // write offsets
  uint32_t *a_i, *a_j;
  uint8_t *a_t;
  uint64_t *f_key;
  uint32_t *f_u, *f_v;
};
// Work plan of the pair passes: particles of sparse cells (one thread each)
// and (cell, 64-particle chunk) units of dense cells (one wave each).
struct PairPlan {
  uint32_t *sparse = nullptr;
  size_t n_sparse = 0;
  uint32_t *ucell = nullptr, *uchunk = nullptr;
  size_t n_units = 0;
};
// dense: cells with at least this many particles take the dense path (one
// wave per 64 home particles), the others the sparse one (a thread each)
void plan_pairs(PairPlan &pl, const uint32_t *cell_of, const uint32_t *cell_start,
                const uint2 *nrange, const uint32_t *n_cells, size_t n, uint32_t dense, Arena &ar,
                hipStream_t s);
// the plan without the sparse homes that found no vulnerable pair in pass 1
void plan_vulnerable(const PairPlan &pl, const uint32_t *cnt_pb, const uint32_t *cnt_pc,
                     PairPlan &out, Arena &ar, hipStream_t s);
void launch_pair_pass1(const PairBufs &b, const PairPlan &pl, hipStream_t s);  // classify, hook
void launch_pair_count(const PairBufs &b, const PairPlan &pl, hipStream_t s);  // filtered counts
void launch_pair_write(const PairBufs &b, const PairPlan &pl, hipStream_t s);  // filtered writes
// slot capacities of the slotted write path from pass 1's class counts: HF
// jobs get pc slots for active pairs and pb slots for forest candidates, VP
// and SC jobs pb + pc slots for active pairs
void pair_slot_caps(const PairBufs &b, uint32_t *cap_a, uint32_t *cap_f, hipStream_t s);
// moves the filled active slots to the front, in home order
void compact_slots(const uint32_t *a_i, const uint32_t *a_j, const uint8_t *a_t,
                   const uint64_t *off_slot, const uint32_t *fill, const uint64_t *off_dense,
                   size_t n, uint32_t *d_i, uint32_t *d_j, uint8_t *d_t, hipStream_t s);
void launch_flatten(uint32_t *par, size_t n, hipStream_t s);
void launch_labels(const uint32_t *root, const float4 *pos, const int64_t *p_off, int njobs,
                   size_t n, uint32_t *minid, int32_t *lab_global, hipStream_t s);
// Boruvka minimum spanning forest over candidate edges (keys distinct).
// Returns the number of forest edges appended at f_out_*.
int64_t boruvka(uint64_t *key, uint32_t *u, uint32_t *v, size_t ncand, uint32_t *bpar,
                size_t n, const uint32_t *inv_perm, const int64_t *p_off, int njobs,
                uint32_t *out_i, uint32_t *out_j, uint8_t *out_t, Arena &ar, hipStream_t s);

// pgd.hip
// Iterates of the PGD loop: one packed record of x, y, z float64 per
// editable row (24 bytes: the step streams rows, and a quarter less per row
// beat the aligned 32-byte records on every workload measured).
constexpr int kPStride = 3;
__device__ inline void load_p(const double *P, size_t i, double &x, double &y, double &z) {
  const double *p = P + (size_t)kPStride * i;
  x = p[0];
  y = p[1];
  z = p[2];
}
__device__ inline void store_p(double *P, size_t i, double x, double y, double z) {
  double *p = P + (size_t)kPStride * i;
  p[0] = x;
  p[1] = y;
  p[2] = z;
}
struct PgdBufs {
  const JobDev *jobs;
  JobLoop *loop;
  const int64_t *e_off;   // [njobs+1] editable rows per job
  const int64_t *tile_off;  // [njobs+1] first 64-row tile of each job
  int64_t ntiles;
  int njobs;
  size_t ne;
  const uint32_t *row_ptr, *col;
  size_t ninc;            // incidences: twice the active pairs
  double *P0, *P1;        // [ne][kPStride]: x, y, z of each row
  double *m, *v;          // [3][ne]
  const float *xo;        // [ne][3] original position of each row
  int32_t *n_active;      // device: jobs not done
  // Hot rows (the only rows evaluated after the first step), per job in
  // wl[e_off[j] .. e_off[j] + wl_n[j]); a step processes the first
  // wl_step[j] of them.  hot[e]: 0 cold, 1 hot, 2 hot with its partners
  // marked hot.
  uint32_t *hot;      // [ne]
  uint32_t *wl;       // [ne]
  uint32_t *wl_n;     // [njobs]
  uint32_t *wl_step;  // [njobs]
  uint32_t *wl_id;    // [njobs] leading entries with wl[e_off[j] + i] = e_off[j] + i
  uint64_t *inc_n;    // [njobs] incidences of the rows in wl[0 .. wl_n)
  uint64_t *inc_step; // [njobs] incidences of the rows a step processes
  // violation count of one evaluation: per job, acc_slots partial sums,
  // each on its own 128-byte line (waves add into the slot of their index,
  // so no address takes many atomics)
  unsigned long long *acc;  // [njobs][acc_slots][16]
  int acc_slots;            // power of two
  // float64 loss of one evaluation: one partial per (job, wave) that holds
  // the wave's sum over its tiles of that job, stored (not added), so the
  // sum the finalize kernel forms in slot order is deterministic.  Job j
  // owns slots lp_off[j] .. lp_off[j+1] - 1, min(its tiles, nwaves) of them;
  // the wave that walks tile k of the job (k counted from the job's first
  // tile) uses slot k mod nwaves.
  double *lossp;
  const int64_t *lp_off;  // [njobs+1]
  int nwaves;             // waves of the step grid (blocks * waves per block)
};
// waves of the step grid for ne editable rows (the step launches exactly
// nwaves / 4 blocks of 4 waves), and of the largest grid; a job's loss slots
// are min(its tiles, pgd_max_waves())
int pgd_step_waves(size_t ne);
int pgd_max_waves();

// The groups one step launch walks: each group is the PGD state of one call
// (PgdBufs), its tiles follow the previous group's in the launch's tile
// space, and its jobs' finalize blocks follow the previous group's.  A plain
// call is one group; the served form's shared loop holds several.
constexpr int kMaxGroups = 64;
constexpr int kMaxGroupJobs = 4096;  // jobs of all groups of the shared loop
struct PgdGroups {
  int32_t ngroups;
  int32_t pad;
  int64_t tile_base[kMaxGroups + 1];
  int32_t job_base[kMaxGroups + 1];
  int32_t active[kMaxGroups];  // shared loop: the groups' not-done job counts
  PgdBufs g[kMaxGroups];
};
// a_k (threshold index per pair) may be NULL; when set it is the last key
void sort_pairs(uint32_t *a_i, uint32_t *a_j, uint8_t *a_t, uint8_t *a_k, size_t na,
                const float4 *pos, int id_bits, Arena &ar, hipStream_t s);
// multi-threshold calls: pairs of job k > 0 move to job 0's particle with the
// same job-local index; a_k[p] receives the job index
void remap_thresholds(uint32_t *a_i, uint32_t *a_j, size_t na, const float4 *pos,
                      const uint32_t *inv_perm, const int64_t *p_off, int njobs, uint8_t *a_k,
                      hipStream_t s);
void mark_editable(const uint32_t *a_i, const uint32_t *a_j, size_t na, size_t n, uint8_t *is_e,
                   uint32_t *eid, uint32_t *ne_dev, Arena &ar, hipStream_t s);
void list_editable(const uint8_t *is_e, const uint32_t *eid, size_t n, uint32_t *e_list,
                   hipStream_t s);
// reorders the editable rows (job-major, then Morton order of their cells);
// e_list and eid are updated in place
void order_rows(uint32_t *e_list, size_t ne, uint32_t *eid, const float4 *pos, const JobDev *jobs,
                const int64_t *p_off, int njobs, Arena &ar, hipStream_t s);
// col entries: partner row | kColPc for created pairs | threshold << kColThrShift;
// every row in increasing (partner's original index, threshold): by a
// stable sort of pairs already in that order (pairs_sorted), else by a rank
// within each row
void build_csr(const uint32_t *a_i, const uint32_t *a_j, const uint8_t *a_t, const uint8_t *a_k,
               size_t na, const uint32_t *eid, uint32_t ne, const uint32_t *e_list,
               const float4 *pos, bool pairs_sorted, uint32_t *row_ptr, uint32_t *col, Arena &ar,
               hipStream_t s);
void launch_pgd_init(const uint32_t *e_list, size_t ne, const float4 *pos, const float4 *rec,
                     double *P0, float *xo, double *m, double *v, hipStream_t s);
// worklist of the first step: every row; no row hot yet
void launch_hot_init(const PgdBufs &b, hipStream_t s);
// After the first step: renumbers each job's rows so that its hot rows come
// first (both groups keep their order).  The row arrays, the CSR (partner
// order within a row unchanged) and the row -> particle list are permuted
// into new buffers, and the worklist becomes the hot rows.
void renumber_hot(PgdBufs &b, uint32_t *&e_list, Arena &ar, hipStream_t s);
void launch_loop_init(const JobDev *jobs, JobLoop *loop, int njobs, int32_t *n_active,
                      hipStream_t s);
// one step (and its finalize) over the groups of the device table g; the
// host copy h gives the launch sizes of a plain call (one group)
void launch_pgd_step(const PgdGroups *g, const PgdBufs &h, hipStream_t s);
void launch_pgd_finalize(const PgdGroups *g, const PgdBufs &h, hipStream_t s);
// the shared loop's launches: the largest grid, kMaxGroupJobs finalize blocks
void launch_pgd_step_shared(const PgdGroups *g, hipStream_t s);
void launch_pgd_finalize_shared(const PgdGroups *g, hipStream_t s);

// encode.hip
struct EncBufs {
  const JobDev *jobs;
  const JobLoop *loop;
  const int64_t *p_off;
  const int64_t *e_off;
  int njobs;
  size_t ne, n;
  const uint32_t *e_list;
  const float4 *pos, *rec;
  const double *P0, *P1;   // [ne][kPStride]
  uint8_t *flag8;          // [n] global original order
  uint32_t *fpos;          // exclusive scan of flag8
  uint16_t *sym;           // symbols
  const uint64_t *sym_off; // [njobs+1] first symbol of each job
  uint32_t *hist;          // [njobs][65536]
  double *debug;           // optional [3][n] global original order
};
void launch_edit_flags(const EncBufs &b, hipStream_t s);
// fstart[j]: flagged particles before job j in the global order
void launch_edit_codes(const EncBufs &b, const uint32_t *fstart, hipStream_t s);
// per-job histograms [njobs][65536] of the symbols
void symbol_histogram(const uint16_t *sym, size_t nsym, const uint64_t *sym_off, int njobs,
                      uint32_t *hist, Arena &ar, hipStream_t s);
void launch_flag_bytes(const uint8_t *flag8, const int64_t *p_off, const uint64_t *fb_off,
                       int njobs, size_t nbytes, uint8_t *bytes, hipStream_t s);
void launch_sym_lengths(const uint16_t *sym, size_t nsym, const uint64_t *sym_off, int njobs,
                        const uint32_t *table, uint32_t *len, hipStream_t s);
void launch_pack_bits(const uint16_t *sym, size_t nsym, const uint64_t *sym_off, int njobs,
                      const uint32_t *table, const uint64_t *bitpos, const uint64_t *job_bit0,
                      const uint64_t *job_word0, uint32_t *words, hipStream_t s);
void launch_debug_xyz(const EncBufs &b, hipStream_t s);

}  // namespace pcc
