// Editable set, constraint incidence lists and the fused PGD step
// (Alg. 1; tightened loss Eq. 3; Adam, Sec. 4.2; box of Eq. 2).
//
// The active pairs become a compressed-row incidence list over the editable
// particles E: row e lists (partner, type) for every active pair of e, in a
// deterministic order (a stable sort of the pair list by row).  One thread
// owns one row: it gathers the partner positions, sums the hinge gradient of
// its own constraints in float64 (no atomics on floats), applies Adam and the
// clamp into the box of half width xi' around the original position, and
// writes the next iterate into the other buffer.  Violations and the loss of
// the current iterate are counted once per pair (in the row with the smaller
// index) into per-job integer accumulators, so convergence decisions and the
// trajectory are bitwise reproducible.
#include "kernels.hpp"

#include <algorithm>

namespace pcc {

// ----------------------------------------------------------------------------
// editable set and CSR
// ----------------------------------------------------------------------------
__global__ void k_mark_e(const uint32_t *a_i, const uint32_t *a_j, size_t na, uint8_t *is_e) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < na;
       p += (size_t)gridDim.x * blockDim.x) {
    is_e[a_i[p]] = 1;
    is_e[a_j[p]] = 1;
  }
}

void mark_editable(const uint32_t *a_i, const uint32_t *a_j, size_t na, size_t n, uint8_t *is_e,
                   uint32_t *eid, uint32_t *ne_dev, Arena &ar, hipStream_t s) {
  fill_u8(is_e, 0, n, s);
  if (na) k_mark_e<<<blocks_for(na, 256, 65536), 256, 0, s>>>(a_i, a_j, na, is_e);
  scan_u8_u32(is_e, eid, n, ne_dev, ar, s);
}

__global__ void k_e_list(const uint8_t *is_e, const uint32_t *eid, size_t n, uint32_t *e_list) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x)
    if (is_e[k]) e_list[eid[k]] = (uint32_t)k;
}

__global__ void k_incid(const uint32_t *a_i, const uint32_t *a_j, const uint8_t *a_t,
                        const uint8_t *a_k, size_t na, const uint32_t *eid, uint32_t *keys,
                        uint32_t *vals) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < na;
       p += (size_t)gridDim.x * blockDim.x) {
    const uint32_t ri = eid[a_i[p]], rj = eid[a_j[p]];
    const uint32_t t = (a_t[p] == 3 ? kColPc : 0u) |
                       (a_k ? (uint32_t)a_k[p] << kColThrShift : 0u);
    keys[2 * p] = ri;
    vals[2 * p] = rj | t;
    keys[2 * p + 1] = rj;
    vals[2 * p + 1] = ri | t;
  }
}

__global__ void k_row_ptr(const uint32_t *keys, size_t m, uint32_t ne, uint32_t *row_ptr) {
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < m;
       q += (size_t)gridDim.x * blockDim.x) {
    if (q == 0 || keys[q] != keys[q - 1]) row_ptr[keys[q]] = (uint32_t)q;
    if (q == m - 1) row_ptr[ne] = (uint32_t)m;
  }
}

static int bits_for(uint64_t v) {
  int b = 0;
  while (b < 32 && (v >> b) != 0) ++b;
  return b;
}

// keys of the active pairs: job-local indices of their two ends
__global__ void k_pair_keys(const uint32_t *a_i, const uint32_t *a_j, size_t na, const float4 *pos,
                            uint32_t *lo, uint32_t *hi, uint32_t *idx) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < na;
       p += (size_t)gridDim.x * blockDim.x) {
    const uint32_t a = __float_as_uint(pos[a_i[p]].w), b = __float_as_uint(pos[a_j[p]].w);
    lo[p] = a < b ? a : b;
    hi[p] = a < b ? b : a;
    idx[p] = (uint32_t)p;
  }
}
__global__ void k_take_u32(const uint32_t *src, const uint32_t *idx, size_t m, uint32_t *dst) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < m;
       p += (size_t)gridDim.x * blockDim.x)
    dst[p] = src[idx[p]];
}
__global__ void k_take_u8_as_u32(const uint8_t *src, const uint32_t *idx, size_t m, uint32_t *dst) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < m;
       p += (size_t)gridDim.x * blockDim.x)
    dst[p] = src[idx[p]];
}
__global__ void k_take_pairs(const uint32_t *a_i, const uint32_t *a_j, const uint8_t *a_t,
                             const uint8_t *a_k, const uint32_t *idx, size_t na, uint32_t *b_i,
                             uint32_t *b_j, uint8_t *b_t, uint8_t *b_k) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < na;
       p += (size_t)gridDim.x * blockDim.x) {
    const uint32_t q = idx[p];
    b_i[p] = a_i[q];
    b_j[p] = a_j[q];
    b_t[p] = a_t[q];
    if (a_k) b_k[p] = a_k[q];
  }
}

// Orders the active pairs by (smaller job-local index, larger one, threshold
// index) with stable radix sorts, least significant key first.  The stable
// sort of their incidences by row that follows then leaves every row in
// increasing partner index (then threshold): the order in which the gradient
// of each particle is summed.
void sort_pairs(uint32_t *a_i, uint32_t *a_j, uint8_t *a_t, uint8_t *a_k, size_t na,
                const float4 *pos, int id_bits, Arena &ar, hipStream_t s) {
  if (na < 2) return;
  uint32_t *lo = ar.get<uint32_t>(na), *hi = ar.get<uint32_t>(na), *idx = ar.get<uint32_t>(na);
  uint32_t *key = ar.get<uint32_t>(na);
  const int nb = blocks_for(na, 256, 65536);
  k_pair_keys<<<nb, 256, 0, s>>>(a_i, a_j, na, pos, lo, hi, idx);
  if (a_k) {
    k_take_u8_as_u32<<<nb, 256, 0, s>>>(a_k, idx, na, key);
    radix_sort_u32(key, idx, na, 3, ar, s);
  }
  k_take_u32<<<nb, 256, 0, s>>>(hi, idx, na, key);
  radix_sort_u32(key, idx, na, id_bits, ar, s);
  k_take_u32<<<nb, 256, 0, s>>>(lo, idx, na, key);
  radix_sort_u32(key, idx, na, id_bits, ar, s);
  uint32_t *b_i = ar.get<uint32_t>(na), *b_j = ar.get<uint32_t>(na);
  uint8_t *b_t = ar.get<uint8_t>(na), *b_k = a_k ? ar.get<uint8_t>(na) : nullptr;
  k_take_pairs<<<nb, 256, 0, s>>>(a_i, a_j, a_t, a_k, idx, na, b_i, b_j, b_t, b_k);
  PCC_HIP(hipMemcpyAsync(a_i, b_i, na * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
  PCC_HIP(hipMemcpyAsync(a_j, b_j, na * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
  PCC_HIP(hipMemcpyAsync(a_t, b_t, na, hipMemcpyDeviceToDevice, s));
  if (a_k) PCC_HIP(hipMemcpyAsync(a_k, b_k, na, hipMemcpyDeviceToDevice, s));
}

// Multi-threshold correction: the jobs of the call are the thresholds of one
// snapshot.  Pairs selected for threshold k > 0 are moved into threshold 0's
// particles (same original index) and tagged with k.
__global__ void k_thr_remap(uint32_t *a_i, uint32_t *a_j, size_t na, const float4 *pos,
                            const uint32_t *inv_perm, const int64_t *p_off, int njobs,
                            uint8_t *a_k) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < na;
       p += (size_t)gridDim.x * blockDim.x) {
    const uint32_t i = a_i[p], j = a_j[p];
    const int k = job_of(p_off, njobs, (int64_t)i);
    a_k[p] = (uint8_t)k;
    if (k > 0) {
      a_i[p] = inv_perm[p_off[0] + __float_as_uint(pos[i].w)];
      a_j[p] = inv_perm[p_off[0] + __float_as_uint(pos[j].w)];
    }
  }
}

void remap_thresholds(uint32_t *a_i, uint32_t *a_j, size_t na, const float4 *pos,
                      const uint32_t *inv_perm, const int64_t *p_off, int njobs, uint8_t *a_k,
                      hipStream_t s) {
  if (na)
    k_thr_remap<<<blocks_for(na, 256, 65536), 256, 0, s>>>(a_i, a_j, na, pos, inv_perm, p_off,
                                                           njobs, a_k);
}

void list_editable(const uint8_t *is_e, const uint32_t *eid, size_t n, uint32_t *e_list,
                   hipStream_t s) {
  if (n) k_e_list<<<blocks_for(n, 256, 65536), 256, 0, s>>>(is_e, eid, n, e_list);
}

// 10 low bits of x spread to every third bit
__device__ inline uint32_t spread3(uint32_t x) {
  x &= 0x3ffu;
  x = (x | (x << 16)) & 0x030000ffu;
  x = (x | (x << 8)) & 0x0300f00fu;
  x = (x | (x << 4)) & 0x030c30c3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

__device__ inline int64_t cell_of_axis(double x, double origin, double inv_w, int nc, bool periodic) {
  if (nc <= 1) return 0;
  int64_t c = (int64_t)floor((x - origin) * inv_w);
  if (periodic) {
    c %= nc;
    if (c < 0) c += nc;
  } else {
    if (c < 0) c = 0;
    if (c >= nc) c = nc - 1;
  }
  return c;
}

// key of a row: its job in the high bits, then the Morton code of its cell
// (each axis cut to `bits` bits), so that the partners of a row lie near it
// in memory along all three axes
__global__ void k_row_keys(const uint32_t *e_list, size_t ne, const float4 *pos, const JobDev *jobs,
                           const int64_t *p_off, int njobs, int bits, uint32_t *keys,
                           uint32_t *vals) {
  for (size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x; r < ne;
       r += (size_t)gridDim.x * blockDim.x) {
    const uint32_t k = e_list[r];
    const int j = job_of(p_off, njobs, (int64_t)k);
    const JobDev &J = jobs[j];
    const float4 p = pos[k];
    const double xyz[3] = {(double)p.x, (double)p.y, (double)p.z};
    uint32_t m = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int64_t c = cell_of_axis(xyz[a], J.origin[a], J.inv_w[a], J.nc[a], (J.periodic >> a) & 1);
      int need = 0;
      while (need < 31 && ((uint32_t)(J.nc[a] - 1) >> need) != 0) ++need;
      const int sh = need > bits ? need - bits : 0;
      m |= spread3((uint32_t)(c >> sh)) << a;
    }
    keys[r] = ((uint32_t)j << (3 * bits)) | m;
    vals[r] = (uint32_t)r;
  }
}

__global__ void k_row_apply(const uint32_t *old_list, const uint32_t *order, size_t ne,
                            uint32_t *new_list, uint32_t *eid) {
  for (size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x; r < ne;
       r += (size_t)gridDim.x * blockDim.x) {
    const uint32_t k = old_list[order[r]];
    new_list[r] = k;
    eid[k] = (uint32_t)r;
  }
}

void order_rows(uint32_t *e_list, size_t ne, uint32_t *eid, const float4 *pos, const JobDev *jobs,
                const int64_t *p_off, int njobs, Arena &ar, hipStream_t s) {
  if (ne < 2) return;
  const int jb = bits_for(njobs > 1 ? (uint64_t)(njobs - 1) : 0);
  const int bits = std::min(10, (32 - jb) / 3);
  uint32_t *keys = ar.get<uint32_t>(ne), *order = ar.get<uint32_t>(ne);
  uint32_t *old = ar.get<uint32_t>(ne);
  const int nb = blocks_for(ne, 256, 65536);
  k_row_keys<<<nb, 256, 0, s>>>(e_list, ne, pos, jobs, p_off, njobs, bits, keys, order);
  radix_sort_u32(keys, order, ne, jb + 3 * bits, ar, s);
  PCC_HIP(hipMemcpyAsync(old, e_list, ne * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
  k_row_apply<<<nb, 256, 0, s>>>(old, order, ne, e_list, eid);
}

// job-local original index of each row's particle
__global__ void k_row_origs(const uint32_t *e_list, size_t ne, const float4 *pos, uint32_t *orig) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne;
       e += (size_t)gridDim.x * blockDim.x)
    orig[e] = __float_as_uint(pos[e_list[e]].w);
}
// order key of an incidence within its row: the partner's original index,
// then the threshold index
__global__ void k_inc_keys(const uint32_t *col, size_t m, const uint32_t *orig, uint64_t *ikey) {
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < m;
       q += (size_t)gridDim.x * blockDim.x) {
    const uint32_t c = col[q];
    ikey[q] = ((uint64_t)orig[c & kColRow] << 3) | ((c >> kColThrShift) & 7u);
  }
}
// Each incidence goes to its rank among the incidences of its row (keys are
// distinct within a row), so every row ends in order of its keys.
__global__ void k_row_rank(const uint32_t *rows, const uint32_t *row_ptr, const uint64_t *ikey,
                           const uint32_t *col, size_t m, uint32_t *out) {
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < m;
       q += (size_t)gridDim.x * blockDim.x) {
    const uint32_t r = rows[q];
    const uint32_t a = row_ptr[r], b = row_ptr[r + 1];
    const uint64_t k = ikey[q];
    uint32_t rank = 0;
    for (uint32_t t = a; t < b; ++t) rank += ikey[t] < k ? 1u : 0u;
    out[a + rank] = col[q];
  }
}

void build_csr(const uint32_t *a_i, const uint32_t *a_j, const uint8_t *a_t, const uint8_t *a_k,
               size_t na, const uint32_t *eid, uint32_t ne, const uint32_t *e_list,
               const float4 *pos, bool pairs_sorted, uint32_t *row_ptr, uint32_t *col, Arena &ar,
               hipStream_t s) {
  if (ne > kColRow) throw Error(-6, "more than 2^28 editable particles in one call");
  if (!na) {
    fill_u32(row_ptr, 0, (size_t)ne + 1, s);
    return;
  }
  const size_t m = 2 * na;
  if (m > 0xffffffffull) throw Error(-6, "more than 2^31 active pairs in one call");
  uint32_t *keys = ar.get<uint32_t>(m);
  uint32_t *c1 = pairs_sorted ? col : ar.get<uint32_t>(m);
  k_incid<<<blocks_for(na, 256, 65536), 256, 0, s>>>(a_i, a_j, a_t, a_k, na, eid, keys, c1);
  radix_sort_u32(keys, c1, m, bits_for(ne ? ne - 1 : 0), ar, s);
  k_row_ptr<<<blocks_for(m, 256, 65536), 256, 0, s>>>(keys, m, ne, row_ptr);
  if (!pairs_sorted) {
    // the stable sort by row kept the pair list's order inside each row;
    // each row is put in increasing (partner index, threshold) instead
    uint32_t *orig = ar.get<uint32_t>(ne);
    uint64_t *ikey = ar.get<uint64_t>(m);
    k_row_origs<<<blocks_for(ne, 256, 65536), 256, 0, s>>>(e_list, ne, pos, orig);
    k_inc_keys<<<blocks_for(m, 256, 65536), 256, 0, s>>>(c1, m, orig, ikey);
    k_row_rank<<<blocks_for(m, 256, 65536), 256, 0, s>>>(keys, row_ptr, ikey, c1, m, col);
  }
}

__global__ void k_pgd_init(const uint32_t *e_list, size_t ne, const float4 *pos, const float4 *rec,
                           double *P0, float *xo, double *m, double *v) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne;
       e += (size_t)gridDim.x * blockDim.x) {
    const uint32_t k = e_list[e];
    const float4 r = rec[k];
    store_p(P0, e, (double)r.x, (double)r.y, (double)r.z);
    const float4 x = pos[k];
    xo[3 * e] = x.x;
    xo[3 * e + 1] = x.y;
    xo[3 * e + 2] = x.z;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      m[a * ne + e] = 0.0;
      v[a * ne + e] = 0.0;
    }
  }
}

void launch_pgd_init(const uint32_t *e_list, size_t ne, const float4 *pos, const float4 *rec,
                     double *P0, float *xo, double *m, double *v, hipStream_t s) {
  if (ne) k_pgd_init<<<blocks_for(ne, 256, 65536), 256, 0, s>>>(e_list, ne, pos, rec, P0, xo, m, v);
}

__global__ void k_loop_init(const JobDev *jobs, JobLoop *loop, int njobs, int32_t *n_active) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) *n_active = njobs;
  if (j >= njobs) return;
  JobLoop L = {};
  L.bc1 = jobs[j].bc_tab[1].x;
  L.bc2 = jobs[j].bc_tab[1].y;
  loop[j] = L;
}

void launch_loop_init(const JobDev *jobs, JobLoop *loop, int njobs, int32_t *n_active,
                      hipStream_t s) {
  k_loop_init<<<(njobs + 255) / 256, 256, 0, s>>>(jobs, loop, njobs, n_active);
}

// ----------------------------------------------------------------------------
// the fused step
// ----------------------------------------------------------------------------
// Minimum image of a difference on a periodic axis (hL = +inf on an open
// one): d - L above hL, d + L below -hL.  Both candidates are formed and one
// is selected, so the wave does not branch per coordinate.
__device__ inline double wrapd(double d, double L, double hL) {
  const double lo = d - L, hi = d + L;
  return d > hL ? lo : (d < -hL ? hi : d);
}

__device__ inline unsigned long long wsum(unsigned long long v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// float64 sum over the wave by a butterfly: every lane ends with the same
// value (a + b and b + a round alike), formed in a fixed order
__device__ inline double wsum_d(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// wave-level barrier: LDS written by lanes of this wave becomes visible to
// all its lanes
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kPgdWaves = 4;
#ifndef PCC_PGD_MIN_WAVES
#define PCC_PGD_MIN_WAVES 4
#endif
// a persistent grid of PCC_PGD_MIN_WAVES waves per SIMD on the 256 CUs
constexpr int kPgdBlocks = 256 * 4 * PCC_PGD_MIN_WAVES / kPgdWaves;

int pgd_step_waves(size_t ne) { return blocks_for(ne, 64 * kPgdWaves, kPgdBlocks) * kPgdWaves; }
int pgd_max_waves() { return kPgdBlocks * kPgdWaves; }


// group of a tile (or of a finalize block): the last with base <= x
template <typename T>
__device__ inline int group_of(const T *base, int ngroups, int64_t x) {
  int lo = 0, hi = ngroups - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((int64_t)base[mid] <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// The dispatcher hands consecutive blocks to the 8 XCDs in turn, and each
// XCD has its own L2.  Renumbering the blocks so that every XCD holds a
// contiguous range of them makes the tiles it walks at the same time
// neighbours in row (Morton) order, whose partner gathers then share its L2.
__device__ inline int xcd_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  if (nb & 7) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

// flush of a wave's counts for one job: the violation count is summed over
// the wave and added into the wave's counter slot; the loss (per lane) is
// summed over the wave and stored into the job's loss slot of this wave
__device__ inline void flush_counts(const PgdBufs &B, int job, int lslot, int wave_id,
                                    unsigned long long &viol, double &loss) {
  const double sl = wsum_d(loss);
  const unsigned long long sv = wsum(viol);
  if ((threadIdx.x & 63) == 0 && job >= 0) {
    if (sv) {
      const int slot = wave_id & (B.acc_slots - 1);
      atomicAdd(B.acc + ((size_t)job * B.acc_slots + slot) * 16, sv);
    }
    B.lossp[B.lp_off[job] + lslot] = sl;
  }
  viol = 0;
  loss = 0.0;
}

__device__ inline uint64_t dbits(double x) { return (uint64_t)__double_as_longlong(x); }

// Each wave walks tiles of up to 64 rows of one job's worklist (tiles never
// straddle two jobs, so the job and its constants are wave-uniform).
//
// Hot rows.  A row whose constraints are all satisfied, whose Adam moments
// are zero and whose position lies in the box is a fixed point of the step
// bit for bit (zero gradient, zero moments, zero displacement, clamp of a
// point already inside), and stays one while none of its partners moves.
// The first step evaluates every row.  A row that is live in some step
// (moved, had a violated constraint or nonzero moments) becomes hot, and so
// do its partners, once; from then on hot rows are evaluated in every step.
// A cold row has never been live and no partner of it has, so none of its
// distances has changed since the first step: it is still a fixed point
// with no violated pair.  Its position is the same in both buffers.  So the
// iterates, the violation counts and the loss are exactly those of
// evaluating every row in every step.
//
// Evaluation.  The tile's incidences, row after row, go to the lanes 64 at
// a time (a chunk): each lane gathers one partner and evaluates one
// constraint, and the row's own lane adds the violated terms of its row in
// column order, so every gradient is summed in the oracle's order.  Two
// chunks are in flight.  The gradients go through LDS to the Adam step and
// the projection, where lane r takes row r (coalesced row reads and
// writes).  Counts stay in registers until the wave moves to another job or
// finishes.  The partners of the rows that turn hot are marked over 64 runs
// of about equal length at row boundaries: lane L takes the rows whose
// first incidence falls in [L T / 64, (L + 1) T / 64) (T incidences in the
// tile).
__global__ void __launch_bounds__(64 * kPgdWaves, PCC_PGD_MIN_WAVES)
    k_pgd_step(const PgdGroups *__restrict__ G) {
  // LDS of one wave: one struct, so that every access is the wave's base
  // (uniform) plus the lane's or row's offset plus a constant
  struct WaveLds {
    double px[64], py[64], pz[64];  // row positions
    double gx[64], gy[64], gz[64];  // row gradients
    double tx[64], ty[64], tz[64];  // chunked evaluation: one term per lane
    // loss thresholds b -+ delta_t and their squares per linking length of
    // a multi-threshold job
    double thr[4][kMaxThresholds];
    uint32_t vb[65];    // tile offset of each row's first incidence
    uint32_t base[64];  // CSR position of a row's incidence f: base + f
    uint32_t e[64];     // row index
    uint8_t hit[64];    // some constraint of the row is violated
    uint8_t mk[64];     // the row marks its partners hot
  };
  __shared__ WaveLds s_lds[kPgdWaves];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  WaveLds &S = s_lds[w];
  const int64_t nwaves = (int64_t)gridDim.x * kPgdWaves;
  const int wave_id = xcd_block() * kPgdWaves + w;
  unsigned long long viol = 0;
  double loss = 0.0;
  int cgrp = 0;    // group and job whose counts are held in the registers above
  int cjob = -1;
  int cslot = 0;   // this wave's loss slot of that job
  const int ngroups = G->ngroups;
  const int64_t ntiles = G->tile_base[ngroups];
  // the buffers of the group being walked, copied once into (scalar)
  // registers: read through the table for every tile they would cost a
  // chain of scalar loads per tile
  PgdBufs B = G->g[0];
  int64_t gbase = 0;
  for (int64_t tile = wave_id; tile < ntiles; tile += nwaves) {
    const int grp =
        ngroups > 1 ? __builtin_amdgcn_readfirstlane(group_of(G->tile_base, ngroups, tile)) : 0;
    if (grp != cgrp) {
      flush_counts(B, cjob, cslot, wave_id, viol, loss);
      B = G->g[grp];
      gbase = G->tile_base[grp];
      cgrp = grp;
      cjob = -1;
    }
    const int64_t tl = tile - gbase;  // tile within its group
    const int job = __builtin_amdgcn_readfirstlane(job_of(B.tile_off, B.njobs, tl));
    if (B.loop[job].done) continue;
    const int64_t eoff = B.e_off[job];
    const int64_t w0 = (tl - B.tile_off[job]) * 64;  // first worklist entry of the tile
    const int64_t left = (int64_t)B.wl_step[job] - w0;
    if (left <= 0) continue;
    if (job != cjob) {
      flush_counts(B, cjob, cslot, wave_id, viol, loss);
      cjob = job;
      cslot = (int)((tl - B.tile_off[job]) % nwaves);
    }
    const int64_t t_step = B.loop[job].t;
    const int nrow = (int)(left < 64 ? left : 64);
    const bool valid = lane < nrow;
    const JobDev &J = B.jobs[job];
    const int cur = (int)(t_step & 1);
    const double *__restrict__ Pc = cur ? B.P1 : B.P0;
    double *__restrict__ Pn = cur ? B.P0 : B.P1;
    const double L0 = J.L[0], L1 = J.L[1], L2 = J.L[2];
    const double h0 = J.hL[0], h1 = J.hL[1], h2 = J.hL[2];
    const double bm = J.bm, bp = J.bp, bm2 = J.bm2, bp2 = J.bp2;
    const bool multi = J.nthr > 1;
    // the row's position and incidence range go to LDS; its Adam state is
    // loaded after the evaluation (fewer live registers, more waves in
    // flight)
    uint32_t total;
    {
      size_t e = 0;
      uint32_t q0 = 0, len = 0;
      double pex = 0.0, pey = 0.0, pez = 0.0;
      if (valid) {
        e = B.wl[eoff + w0 + lane];
        q0 = B.row_ptr[e];
        len = B.row_ptr[e + 1] - q0;
        load_p(Pc, e, pex, pey, pez);
      }
      uint32_t incl = len;  // inclusive prefix sum of len over the wave
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += y;
      }
      const uint32_t vb = incl - len;
      total = __shfl(incl, 63, kWave);
      S.px[lane] = pex;
      S.py[lane] = pey;
      S.pz[lane] = pez;
      S.gx[lane] = 0.0;
      S.gy[lane] = 0.0;
      S.gz[lane] = 0.0;
      S.hit[lane] = 0;
      S.vb[lane] = vb;
      if (lane == 63) S.vb[64] = total;
      S.base[lane] = q0 - vb;
      S.e[lane] = (uint32_t)e;
    }
    if (multi && lane < 4 * kMaxThresholds) {
      const int a = lane / kMaxThresholds, k = lane % kMaxThresholds;
      const double *src = a == 0 ? J.thr_bm : a == 1 ? J.thr_bp : a == 2 ? J.thr_bm2 : J.thr_bp2;
      S.thr[a][k] = src[k];
    }
    wave_sync();
    // the term of one incidence (column word col, partner position o) in
    // the row at r (index er); a violated pair adds its squared hinge and a
    // count once, in the row of its smaller index
    auto eval = [&](uint32_t col, double ox, double oy, double oz, double rx, double ry,
                    double rz, uint32_t er, double &tx, double &ty, double &tz) -> bool {
      const uint32_t o = col & kColRow;
      const double dx = wrapd(rx - ox, L0, h0);
      const double dy = wrapd(ry - oy, L1, h1);
      const double dz = wrapd(rz - oz, L2, h2);
      const double d2 = (dx * dx + dy * dy) + dz * dz;
      // squared threshold of the constraint (b - delta_t for a potentially
      // broken link, b + delta_t for a potentially created pair): of the
      // job's linking length, or of the constraint's own when several are
      // corrected at once
      const bool created = (col & kColPc) != 0;
      const uint32_t kk = (col >> kColThrShift) & 7u;
      double t2 = created ? bp2 : bm2;
      if (kk) t2 = S.thr[created ? 3 : 2][kk];
      if (!(created ? d2 <= t2 : d2 > t2)) return false;
      double t1 = created ? bp : bm;
      if (kk) t1 = S.thr[created ? 1 : 0][kk];
      const double d = sqrt(d2);
      double h;
      if (!created) {
        // potentially broken: an original link pulled back inside b - delta_t
        h = d - t1;
        // one divide at a time (interleaved divide sequences cost
        // registers, hence occupancy)
        tx = 2.0 * h * (dx / d);
        __builtin_amdgcn_sched_barrier(0);
        ty = 2.0 * h * (dy / d);
        __builtin_amdgcn_sched_barrier(0);
        tz = 2.0 * h * (dz / d);
      } else {
        // potentially created: an original non-link pushed beyond b + delta_t
        h = t1 - d;
        double ux, uy, uz;
        if (d > 0.0) {
          ux = dx / d;
          __builtin_amdgcn_sched_barrier(0);
          uy = dy / d;
          __builtin_amdgcn_sched_barrier(0);
          uz = dz / d;
        } else {
          // coincident points: take the direction of the original pair
          const float *a = B.xo + 3 * (size_t)er, *b = B.xo + 3 * (size_t)o;
          const double ox2 = wrapd((double)a[0] - (double)b[0], L0, h0);
          const double oy2 = wrapd((double)a[1] - (double)b[1], L1, h1);
          const double oz2 = wrapd((double)a[2] - (double)b[2], L2, h2);
          const double od = sqrt((ox2 * ox2 + oy2 * oy2) + oz2 * oz2);
          ux = ox2 / od;
          uy = oy2 / od;
          uz = oz2 / od;
        }
        tx = -(2.0 * h * ux);
        ty = -(2.0 * h * uy);
        tz = -(2.0 * h * uz);
      }
      if (o > er) {
        loss += h * h;
        viol += 1;
      }
      return true;
    };
    auto gather = [&](uint32_t col, double &x, double &y, double &z) {
      load_p(Pc, col & kColRow, x, y, z);
    };
    // this lane's rows [r0, r1) in the balanced split of the tile's
    // incidences (the partner marking below walks them): those whose first
    // incidence lies in [ta, tb)
    const uint32_t ta = (uint32_t)(((uint64_t)lane * total + 63u) / 64u);
    const uint32_t tb = (uint32_t)(((uint64_t)(lane + 1) * total + 63u) / 64u);
    auto first_at = [&](uint32_t t) {
      int lo = 0, hi = nrow;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (S.vb[mid] < t)
          lo = mid + 1;
        else
          hi = mid;
      }
      return lo;
    };
    const int r0 = first_at(ta), r1 = first_at(tb);
    const uint32_t fA = S.vb[r0], fB = S.vb[r1];
    {
      // The tile's incidences are spread over the lanes 64 at a time (one
      // partner gather per lane, two chunks in flight), each lane leaves
      // its term in LDS and the row's own lane adds the violated terms of
      // its row in column order.
      double gx = 0.0, gy = 0.0, gz = 0.0;
      bool hrow = false;
      const uint32_t vb = S.vb[lane], vend = S.vb[lane < 63 ? lane + 1 : 64];
      // row of tile slot q: the last row starting at or before it
      auto locate = [&](uint32_t q, int &r, uint32_t &col) {
        int lo = 0, hi = nrow - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (S.vb[mid] <= q)
            lo = mid;
          else
            hi = mid - 1;
        }
        r = lo;
        col = B.col[S.base[lo] + q];
      };
      int r_nx = 0, r_nx2 = 0;
      uint32_t col_nx = 0, col_nx2 = 0;
      double ax = 0.0, ay = 0.0, az = 0.0;
      if ((uint32_t)lane < total) {
        locate(lane, r_nx, col_nx);
        gather(col_nx, ax, ay, az);
      }
      if ((uint32_t)lane + 64 < total) locate(lane + 64, r_nx2, col_nx2);
      for (uint32_t c0 = 0; c0 < total; c0 += 64) {
        const uint32_t q = c0 + lane;
        double tx = 0.0, ty = 0.0, tz = 0.0;
        bool hit = false;
        const int r = r_nx;
        const uint32_t col = col_nx;
        const double ox = ax, oy = ay, oz = az;
        r_nx = r_nx2;
        col_nx = col_nx2;
        if (q + 64 < total) gather(col_nx, ax, ay, az);
        if (q + 128 < total) locate(q + 128, r_nx2, col_nx2);
        if (q < total) hit = eval(col, ox, oy, oz, S.px[r], S.py[r], S.pz[r], S.e[r], tx, ty, tz);
        const uint64_t hb = __ballot(hit);
        if (hb == 0) continue;  // no term of this chunk is nonzero
        S.tx[lane] = tx;
        S.ty[lane] = ty;
        S.tz[lane] = tz;
        wave_sync();
        // the row's lane adds its violated terms that fall in this chunk, in
        // order (a satisfied constraint's +0.0 would leave the sum unchanged)
        const uint32_t a = vb > c0 ? vb : c0;
        const uint32_t b = vend < c0 + 64 ? vend : c0 + 64;
        if (b > a) {
          const uint32_t wd = b - a;
          const uint64_t mask = (wd >= 64 ? ~0ull : ((1ull << wd) - 1ull)) << (a - c0);
          uint64_t mine = hb & mask;
          hrow |= mine != 0;
          while (mine) {
            const int t = __builtin_ctzll(mine);
            gx += S.tx[t];
            gy += S.ty[t];
            gz += S.tz[t];
            mine &= mine - 1;
          }
        }
        wave_sync();
      }
      if (valid) {
        S.gx[lane] = gx;
        S.gy[lane] = gy;
        S.gz[lane] = gz;
        S.hit[lane] = hrow ? 1 : 0;
      }
    }
    wave_sync();
    bool mark = false;
    if (valid) {
      const size_t e = S.e[lane];
      const uint32_t hotv = B.hot[e];
      const float *x = B.xo + 3 * e;
      double mo[3], vo[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        mo[k] = B.m[(size_t)k * B.ne + e];
        vo[k] = B.v[(size_t)k * B.ne + e];
      }
      const double bc1 = B.loop[job].bc1, bc2 = B.loop[job].bc2;
      // the step's constants, read once: the compiler must assume that the
      // moment stores below may alias the job table, and would load them
      // again (and wait for the load) for every coordinate
      const int opt = J.optimizer;
      const double lr = J.lr, beta1 = J.beta1, beta2 = J.beta2,
                   omb1 = J.one_m_beta1,
                   omb2 = J.one_m_beta2, aeps = J.adam_eps, xip = J.xi_p;
      const double g[3] = {S.gx[lane], S.gy[lane], S.gz[lane]};
      const double p[3] = {S.px[lane], S.py[lane], S.pz[lane]};
      const double xs[3] = {(double)x[0], (double)x[1], (double)x[2]};
      double np[3];
      uint64_t state = 0;
      bool moved = false;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double r;
        if (opt == 1) {
          r = p[k] - lr * g[k];
        } else {
          const size_t ia = (size_t)k * B.ne + e;
          const double m = beta1 * mo[k] + omb1 * g[k];
          const double v = beta2 * vo[k] + omb2 * g[k] * g[k];
          B.m[ia] = m;
          B.v[ia] = v;
          state |= dbits(m) | dbits(v);
          const double mh = m / bc1;
          const double vh = v / bc2;
          r = p[k] - lr * mh / (sqrt(vh) + aeps);
        }
        np[k] = fmin(fmax(r, xs[k] - xip), xs[k] + xip);
        moved |= dbits(np[k]) != dbits(p[k]);
        // one coordinate at a time: interleaving the three divide and
        // square-root sequences costs registers, hence occupancy
        __builtin_amdgcn_sched_barrier(0);
      }
      store_p(Pn, e, np[0], np[1], np[2]);
      // a live row that has not yet done so marks itself and its partners hot
      mark = (moved || S.hit[lane] || state != 0) && hotv != 2;
      if (mark) B.hot[e] = 2;
    }
    if (__ballot(mark)) {
      S.mk[lane] = mark ? 1 : 0;
      wave_sync();
      // the balanced runs, walked in step by every lane (the appends below
      // take a wave-wide ballot)
      unsigned long long run = fB - fA;
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) {
        const unsigned long long y = __shfl_xor(run, d, kWave);
        run = y > run ? y : run;
      }
      int rm = fA < fB ? r0 : 0;
      for (uint32_t k = 0; k < (uint32_t)run; ++k) {
        const uint32_t f = fA + k;
        bool app = false;
        uint32_t o = 0;
        if (f < fB) {
          while (S.vb[rm + 1] <= f) ++rm;
          if (S.mk[rm]) {
            o = B.col[S.base[rm] + f] & kColRow;
            uint32_t cold = 0u;
            // the first marking of a cold row appends it to the worklist
            // (after the first step, which lists every row and is followed
            // by a compaction of the hot ones)
            app = __hip_atomic_compare_exchange_strong(B.hot + o, &cold, 1u, __ATOMIC_RELAXED,
                                                       __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT) &&
                  t_step > 0;
          }
        }
        const uint64_t am = __ballot(app);
        if (am) {
          const unsigned long long deg = app ? B.row_ptr[o + 1] - B.row_ptr[o] : 0u;
          const unsigned long long sdeg = wsum(deg);
          uint32_t base = 0;
          if (lane == 0) {
            base = atomicAdd(B.wl_n + job, (uint32_t)__popcll(am));
            atomicAdd((unsigned long long *)B.inc_n + job, sdeg);
          }
          base = __shfl(base, 0, kWave);
          if (app) B.wl[eoff + base + __popcll(am & ((1ull << lane) - 1ull))] = o;
        }
      }
    }
    wave_sync();  // LDS of this tile is reused by the next one
  }
  flush_counts(B, cjob, cslot, wave_id, viol, loss);
}

// flush of a wave's counts for one job: the violation count (the same in
// every lane) is added into the wave's counter slot; the loss (per lane) is
// summed over the wave and stored into the job's loss slot of this wave
__device__ inline void flush_rows(const PgdBufs &B, int job, int lslot,
                                    unsigned long long &viol, double &loss) {
  const double sl = wsum_d(loss);
  if ((threadIdx.x & 63) == 0 && job >= 0) {
    if (viol) {
      const int slot = (int)((blockIdx.x * kPgdWaves + (threadIdx.x >> 6)) & (B.acc_slots - 1));
      atomicAdd(B.acc + ((size_t)job * B.acc_slots + slot) * 16, viol);
    }
    B.lossp[B.lp_off[job] + lslot] = sl;
  }
  viol = 0;
  loss = 0.0;
}

// The step of a plain call (one group, passed by value).  Each wave walks
// tiles of up to 64 rows of one job's worklist (tiles never straddle two
// jobs, so the job and its constants are wave-uniform).
//
// Hot rows.  A row whose constraints are all satisfied, whose Adam moments
// are zero and whose position lies in the box is a fixed point of the step
// bit for bit (zero gradient, zero moments, zero displacement, clamp of a
// point already inside), and stays one while none of its partners moves.
// The first step evaluates every row.  A row that is live in some step
// (moved, had a violated constraint or nonzero moments) becomes hot, and so
// do its partners, once; from then on hot rows are evaluated in every step.
// A cold row has never been live and no partner of it has, so none of its
// distances has changed since the first step: it is still a fixed point
// with no violated pair.  Its position is the same in both buffers.  So the
// iterates, the violation counts and the loss are exactly those of
// evaluating every row in every step.
//
// The incidences of the tile's rows are concatenated and spread over the 64
// lanes, 64 at a time: each lane gathers one partner, evaluates one
// constraint and leaves its gradient term in LDS; then each row's owner
// lane adds the terms of its row in column order (increasing partner index).
// Finally every row takes the Adam step and the projection.  Counts stay in
// registers until the wave moves to another job or finishes.
#ifndef PCC_PGD_MIN_WAVES
#define PCC_PGD_MIN_WAVES 4
#endif
__global__ void __launch_bounds__(64 * kPgdWaves, PCC_PGD_MIN_WAVES) k_pgd_rows(PgdBufs B) {
  // positions of the tile's rows, one array per axis: lanes read rows at
  // random, and 8-byte entries spread them over the LDS banks
  __shared__ double s_px[kPgdWaves][64], s_py[kPgdWaves][64], s_pz[kPgdWaves][64];
  __shared__ double s_term[kPgdWaves][3][64];
  __shared__ uint32_t s_rp[kPgdWaves][64];  // first incidence of each row in the CSR
  __shared__ uint32_t s_vb[kPgdWaves][64];  // first slot of each row in the tile's work list
  __shared__ uint32_t s_e[kPgdWaves][64];   // row index
  __shared__ uint8_t s_mk[kPgdWaves][64];   // the row marks its partners hot
  __shared__ int8_t s_own[kPgdWaves][64];   // row starting at each slot of a chunk
  // loss thresholds b -+ delta_t and their squares per linking length of a
  // multi-threshold job (read from LDS: a memory load in the evaluation
  // would make the gathers already in flight complete first)
  __shared__ double s_thr[kPgdWaves][4][kMaxThresholds];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t nwaves = (int64_t)gridDim.x * kPgdWaves;
  unsigned long long viol = 0;
  double loss = 0.0;
  int cjob = -1;   // job whose counts are held in the registers above
  int cslot = 0;   // this wave's loss slot of that job
  for (int64_t tile = (int64_t)blockIdx.x * kPgdWaves + w; tile < B.ntiles; tile += nwaves) {
    const int job = __builtin_amdgcn_readfirstlane(job_of(B.tile_off, B.njobs, tile));
    if (B.loop[job].done) continue;
    const int64_t eoff = B.e_off[job];
    const int64_t w0 = (tile - B.tile_off[job]) * 64;  // first worklist entry of the tile
    const int64_t left = (int64_t)B.wl_step[job] - w0;
    if (left <= 0) continue;
    const uint32_t wl_ident = B.wl_id[job];
    if (job != cjob) {
      flush_rows(B, cjob, cslot, viol, loss);
      cjob = job;
      cslot = (int)((tile - B.tile_off[job]) % nwaves);
    }
    const int64_t t_step = B.loop[job].t;
    const int nrow = (int)(left < 64 ? left : 64);
    const bool valid = lane < nrow;
    const JobDev &J = B.jobs[job];
    const int cur = (int)(t_step & 1);
    const double *__restrict__ Pc = cur ? B.P1 : B.P0;
    double *__restrict__ Pn = cur ? B.P0 : B.P1;
    const double L0 = J.L[0], L1 = J.L[1], L2 = J.L[2];
    const double h0 = J.hL[0], h1 = J.hL[1], h2 = J.hL[2];
    const double bm = J.bm, bp = J.bp, bm2 = J.bm2, bp2 = J.bp2;
    // the row's position and incidence range; its Adam state is loaded
    // after the gathers (fewer live registers, more waves in flight)
    size_t e = 0;
    uint32_t q0 = 0, len = 0;
    double4 pe = make_double4(0.0, 0.0, 0.0, 0.0);
    if (valid) {
      // the worklist's leading entries are the identity (every row before
      // the first step, the renumbered hot rows after it): no read
      const int64_t wi = w0 + lane;
      e = wi < (int64_t)wl_ident ? (size_t)(eoff + wi) : (size_t)B.wl[eoff + wi];
      q0 = B.row_ptr[e];
      len = B.row_ptr[e + 1] - q0;
      load_p(Pc, e, pe.x, pe.y, pe.z);
    }
    uint32_t incl = len;  // inclusive prefix sum of len over the wave
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(incl, d, kWave);
      if (lane >= d) incl += y;
    }
    const uint32_t vb = incl - len, total = __shfl(incl, 63, kWave);
    s_px[w][lane] = pe.x;
    s_py[w][lane] = pe.y;
    s_pz[w][lane] = pe.z;
    s_rp[w][lane] = q0;
    s_vb[w][lane] = vb;
    s_e[w][lane] = (uint32_t)e;
    if (J.nthr > 1 && lane < 4 * kMaxThresholds) {
      const int a = lane / kMaxThresholds, k = lane % kMaxThresholds;
      const double *src = a == 0 ? J.thr_bm : a == 1 ? J.thr_bp : a == 2 ? J.thr_bm2 : J.thr_bp2;
      s_thr[w][a][k] = src[k];
    }
    wave_sync();
    double gx = 0.0, gy = 0.0, gz = 0.0;
    bool hrow = false;  // some constraint of the row is violated
    // Owner row of slot q = c + lane of the chunk starting at slot c (the
    // last row starting at or before q) and its column entry.  The rows
    // that start inside the chunk mark their first slot, and a running
    // maximum over the lanes, seeded with the owner of the slot before the
    // chunk (carry), gives every slot its row; chunks are located in order.
    // Each chunk loads the next chunk's entries before it waits for its own
    // gathers.
    int carry = 0;
    auto locate = [&](uint32_t c, int &r, uint32_t &col) {
      s_own[w][lane] = -1;
      wave_sync();
      if (len > 0 && vb >= c && vb < c + 64) s_own[w][vb - c] = (int8_t)lane;
      wave_sync();
      int o = s_own[w][lane];
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(o, d, kWave);
        if (lane >= d) o = t > o ? t : o;
      }
      o = carry > o ? carry : o;
      carry = __shfl(o, 63, kWave);
      r = o;
      const uint32_t q = c + lane;
      col = q < total ? B.col[s_rp[w][o] + (q - s_vb[w][o])] : 0u;
    };
    // two-deep pipeline: while chunk c is evaluated, the partner gather of
    // chunk c + 1 and the column entries of chunk c + 2 are in flight
    auto gather = [&](uint32_t col) {
      const double *pp = Pc + (size_t)kPStride * (col & kColRow);
      return make_double3(pp[0], pp[1], pp[2]);
    };
    int r_nx = 0, r_nx2 = 0;
    uint32_t col_nx = 0, col_nx2 = 0;
    double3 po_nx = make_double3(0.0, 0.0, 0.0);
    if (total > 0) {
      locate(0, r_nx, col_nx);
      if ((uint32_t)lane < total) po_nx = gather(col_nx);
    }
    if (total > 64) locate(64, r_nx2, col_nx2);
    for (uint32_t c0 = 0; c0 < total; c0 += 64) {
      const uint32_t q = c0 + lane;
      double tx = 0.0, ty = 0.0, tz = 0.0;
      bool hit = false, hit_once = false;
      const int r = r_nx;
      const uint32_t col = col_nx;
      const double3 po = po_nx;
      r_nx = r_nx2;
      col_nx = col_nx2;
      if (q + 64 < total) po_nx = gather(col_nx);
      if (c0 + 128 < total) locate(c0 + 128, r_nx2, col_nx2);
      if (q < total) {
        const uint32_t o = col & kColRow;
        const uint32_t er = s_e[w][r];
        const double dx = wrapd(s_px[w][r] - po.x, L0, h0);
        const double dy = wrapd(s_py[w][r] - po.y, L1, h1);
        const double dz = wrapd(s_pz[w][r] - po.z, L2, h2);
        const double d2 = (dx * dx + dy * dy) + dz * dz;
        // squared threshold of the constraint (b - delta_t for a potentially
        // broken link, b + delta_t for a potentially created pair): of the
        // job's linking length, or of the constraint's own when several are
        // corrected at once
        const bool created = (col & kColPc) != 0;
        const uint32_t kk = (col >> kColThrShift) & 7u;
        double t2 = created ? bp2 : bm2;
        if (kk) t2 = s_thr[w][created ? 3 : 2][kk];
        double h = 0.0;
        if (created ? d2 <= t2 : d2 > t2) {
          double t1 = created ? bp : bm;
          if (kk) t1 = s_thr[w][created ? 1 : 0][kk];
          const double d = sqrt(d2);
          if (!created) {
            // potentially broken: an original link pulled back inside b - delta_t
            h = d - t1;
            tx = 2.0 * h * (dx / d);
            ty = 2.0 * h * (dy / d);
            tz = 2.0 * h * (dz / d);
          } else {
            // potentially created: an original non-link pushed beyond b + delta_t
            h = t1 - d;
            double ux, uy, uz;
            if (d > 0.0) {
              ux = dx / d;
              uy = dy / d;
              uz = dz / d;
            } else {
              // coincident points: take the direction of the original pair
              const float *a = B.xo + 3 * (size_t)er, *b = B.xo + 3 * (size_t)o;
              const double ox = wrapd((double)a[0] - (double)b[0], L0, h0);
              const double oy = wrapd((double)a[1] - (double)b[1], L1, h1);
              const double oz = wrapd((double)a[2] - (double)b[2], L2, h2);
              const double od = sqrt((ox * ox + oy * oy) + oz * oz);
              ux = ox / od;
              uy = oy / od;
              uz = oz / od;
            }
            tx = -(2.0 * h * ux);
            ty = -(2.0 * h * uy);
            tz = -(2.0 * h * uz);
          }
          hit = true;
        }
        if (hit && o > er) loss += h * h;
        hit_once = hit && o > er;
      }
      const uint64_t hb = __ballot(hit);
      viol += (unsigned)__popcll(__ballot(hit_once));
      if (hb == 0) continue;  // no term of this chunk is nonzero
      s_term[w][0][lane] = tx;
      s_term[w][1][lane] = ty;
      s_term[w][2][lane] = tz;
      wave_sync();
      // The owner adds the violated terms of its row that fall in this
      // chunk, in order.  A satisfied constraint contributes +0.0, which
      // leaves a running sum that starts at +0.0 bitwise unchanged, so
      // skipping it gives the same sum as adding every term.
      const uint32_t a = vb > c0 ? vb : c0;
      const uint32_t b = vb + len < c0 + 64 ? vb + len : c0 + 64;
      if (b > a) {
        const uint32_t wd = b - a;
        const uint64_t mask = (wd >= 64 ? ~0ull : ((1ull << wd) - 1ull)) << (a - c0);
        uint64_t mine = hb & mask;
        hrow |= mine != 0;
        while (mine) {
          const int t = __builtin_ctzll(mine);
          gx += s_term[w][0][t];
          gy += s_term[w][1][t];
          gz += s_term[w][2][t];
          mine &= mine - 1;
        }
      }
      wave_sync();
    }
    bool mark = false;
    if (valid) {
      const uint32_t hotv = B.hot[e];
      const float *x = B.xo + 3 * e;
      double mo[3], vo[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        mo[k] = B.m[(size_t)k * B.ne + e];
        vo[k] = B.v[(size_t)k * B.ne + e];
      }
      const double bc1 = B.loop[job].bc1, bc2 = B.loop[job].bc2;
      // the step's constants, read once: the compiler must assume that the
      // moment stores below may alias the job table, and would load them
      // again (and wait for the load) for every coordinate
      const int opt = J.optimizer;
      const double lr = J.lr, beta1 = J.beta1, beta2 = J.beta2,
                   omb1 = J.one_m_beta1,
                   omb2 = J.one_m_beta2, aeps = J.adam_eps, xip = J.xi_p;
      const double g[3] = {gx, gy, gz};
      const double p[3] = {s_px[w][lane], s_py[w][lane], s_pz[w][lane]};
      const double xs[3] = {(double)x[0], (double)x[1], (double)x[2]};
      double np[3];
      uint64_t state = 0;
      bool moved = false;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double r;
        if (opt == 1) {
          r = p[k] - lr * g[k];
        } else {
          const size_t ia = (size_t)k * B.ne + e;
          const double m = beta1 * mo[k] + omb1 * g[k];
          const double v = beta2 * vo[k] + omb2 * g[k] * g[k];
          B.m[ia] = m;
          B.v[ia] = v;
          state |= dbits(m) | dbits(v);
          const double mh = m / bc1;
          const double vh = v / bc2;
          r = p[k] - lr * mh / (sqrt(vh) + aeps);
        }
        np[k] = fmin(fmax(r, xs[k] - xip), xs[k] + xip);
        moved |= dbits(np[k]) != dbits(p[k]);
        // one coordinate at a time: interleaving the three divide and
        // square-root sequences costs registers, hence occupancy
        __builtin_amdgcn_sched_barrier(0);
      }
      store_p(Pn, e, np[0], np[1], np[2]);
      // a live row that has not yet done so marks itself and its partners hot
      mark = (moved || hrow || state != 0) && hotv != 2;
      if (mark) B.hot[e] = 2;
    }
    if (__ballot(mark)) {
      s_mk[w][lane] = mark ? 1 : 0;
      wave_sync();
      for (uint32_t c0 = 0; c0 < total; c0 += 64) {
        const uint32_t q = c0 + lane;
        bool app = false;
        uint32_t o = 0;
        if (q < total) {
          int lo = 0, hi = nrow - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_vb[w][mid] <= q)
              lo = mid;
            else
              hi = mid - 1;
          }
          if (s_mk[w][lo]) {
            o = B.col[s_rp[w][lo] + (q - s_vb[w][lo])] & kColRow;
            uint32_t cold = 0u;
            // the first marking of a cold row appends it to the worklist
            // (after the first step, which lists every row and is followed
            // by a compaction of the hot ones)
            app = __hip_atomic_compare_exchange_strong(B.hot + o, &cold, 1u, __ATOMIC_RELAXED,
                                                       __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT) &&
                  t_step > 0;
          }
        }
        const uint64_t am = __ballot(app);
        if (am) {
          const unsigned long long deg = app ? B.row_ptr[o + 1] - B.row_ptr[o] : 0u;
          const unsigned long long sdeg = wsum(deg);
          uint32_t base = 0;
          if (lane == 0) {
            base = atomicAdd(B.wl_n + job, (uint32_t)__popcll(am));
            atomicAdd((unsigned long long *)B.inc_n + job, sdeg);
          }
          base = __shfl(base, 0, kWave);
          if (app) B.wl[eoff + base + __popcll(am & ((1ull << lane) - 1ull))] = o;
        }
      }
    }
    wave_sync();  // LDS of this tile is reused by the next one
  }
  flush_rows(B, cjob, cslot, viol, loss);
}

__global__ void k_hot_init(PgdBufs B, size_t n) {
  const size_t nacc = (size_t)B.njobs * B.acc_slots * 16;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    if (i < B.ne) {
      B.hot[i] = 0;
      B.wl[i] = (uint32_t)i;
    }
    if (i < (size_t)B.njobs) {
      B.wl_n[i] = 0;
      B.wl_step[i] = (uint32_t)(B.e_off[i + 1] - B.e_off[i]);
      B.wl_id[i] = B.wl_step[i];
      B.inc_n[i] = 0;
      B.inc_step[i] = B.ne ? (uint64_t)B.row_ptr[B.e_off[i + 1]] - B.row_ptr[B.e_off[i]] : 0;
    }
    if (i < nacc) B.acc[i] = 0;
  }
}

void launch_hot_init(const PgdBufs &b, hipStream_t s) {
  const size_t n = std::max(std::max(b.ne, (size_t)b.njobs), (size_t)b.njobs * b.acc_slots * 16);
  if (n) k_hot_init<<<blocks_for(n, 256, 65536), 256, 0, s>>>(b, n);
}

__global__ void k_hot_flags(const uint32_t *hot, size_t ne, uint8_t *f) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ne;
       i += (size_t)gridDim.x * blockDim.x)
    f[i] = hot[i] != 0;
}

// new index of each row: the job's hot rows first, then its cold rows
__global__ void k_new_ids(const uint8_t *f, const uint32_t *pos, const uint32_t *total, size_t ne,
                          const int64_t *e_off, int njobs, uint32_t *new_id) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne;
       e += (size_t)gridDim.x * blockDim.x) {
    const int j = job_of(e_off, njobs, (int64_t)e);
    const int64_t s = e_off[j], t = e_off[j + 1];
    const uint32_t hs = pos[s], ht = t < (int64_t)ne ? pos[t] : *total;
    const uint32_t before = pos[e] - hs;  // hot rows of the job before e
    new_id[e] = f[e] ? (uint32_t)s + before
                     : (uint32_t)s + (ht - hs) + ((uint32_t)(e - s) - before);
  }
}

struct RowPerm {
  const uint32_t *new_id;
  const double *P0, *P1;
  const double *m, *v;
  const float *xo;
  const uint32_t *hot, *e_list, *row_ptr;
  double *nP0, *nP1;
  double *nm, *nv;
  float *nxo;
  uint32_t *nhot, *ne_list, *nlen, *wl;
};

__global__ void k_permute_rows(RowPerm R, size_t ne) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne;
       e += (size_t)gridDim.x * blockDim.x) {
    const uint32_t r = R.new_id[e];
#pragma unroll
    for (int k = 0; k < kPStride; ++k) {
      R.nP0[(size_t)kPStride * r + k] = R.P0[(size_t)kPStride * e + k];
      R.nP1[(size_t)kPStride * r + k] = R.P1[(size_t)kPStride * e + k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) R.nxo[3 * (size_t)r + k] = R.xo[3 * e + k];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      R.nm[(size_t)k * ne + r] = R.m[(size_t)k * ne + e];
      R.nv[(size_t)k * ne + r] = R.v[(size_t)k * ne + e];
    }
    R.nhot[r] = R.hot[e];
    R.ne_list[r] = R.e_list[e];
    R.nlen[r] = R.row_ptr[e + 1] - R.row_ptr[e];
    R.wl[e] = (uint32_t)e;
  }
}

__global__ void k_permute_cols(const uint32_t *new_id, const uint32_t *row_ptr, const uint32_t *col,
                               const uint32_t *nrow_ptr, size_t ne, uint32_t *ncol) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne;
       e += (size_t)gridDim.x * blockDim.x) {
    const uint32_t a = row_ptr[e], b = row_ptr[e + 1], d = nrow_ptr[new_id[e]];
    for (uint32_t q = a; q < b; ++q) {
      const uint32_t c = col[q];
      ncol[d + (q - a)] = new_id[c & kColRow] | (c & ~kColRow);
    }
  }
}

__global__ void k_hot_counts(const uint32_t *pos, const uint32_t *total, const uint32_t *nrow_ptr,
                             const int64_t *e_off, int njobs, size_t ne, uint32_t *wl_n,
                             uint32_t *wl_step, uint32_t *wl_id, uint64_t *inc_n,
                             uint64_t *inc_step) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= njobs) return;
  const int64_t s = e_off[j], t = e_off[j + 1];
  const uint32_t a = s < (int64_t)ne ? pos[s] : *total, b = t < (int64_t)ne ? pos[t] : *total;
  wl_n[j] = b - a;
  wl_step[j] = b - a;
  wl_id[j] = b - a;  // the renumbering leaves the worklist the identity
  // the hot rows are now e_off[j] .. e_off[j] + (b - a) - 1
  const uint64_t inc = (uint64_t)nrow_ptr[s + (b - a)] - nrow_ptr[s];
  inc_n[j] = inc;
  inc_step[j] = inc;
}

void renumber_hot(PgdBufs &b, uint32_t *&e_list, Arena &ar, hipStream_t s) {
  const size_t ne = b.ne;
  if (!ne) return;
  uint8_t *f = ar.get<uint8_t>(ne);
  uint32_t *pos = ar.get<uint32_t>(ne), *total = ar.get<uint32_t>(1);
  uint32_t *new_id = ar.get<uint32_t>(ne);
  const int nb = blocks_for(ne, 256, 65536);
  k_hot_flags<<<nb, 256, 0, s>>>(b.hot, ne, f);
  scan_u8_u32(f, pos, ne, total, ar, s);
  k_new_ids<<<nb, 256, 0, s>>>(f, pos, total, ne, b.e_off, b.njobs, new_id);
  RowPerm R;
  R.new_id = new_id;
  R.P0 = b.P0;
  R.P1 = b.P1;
  R.m = b.m;
  R.v = b.v;
  R.xo = b.xo;
  R.hot = b.hot;
  R.e_list = e_list;
  R.row_ptr = b.row_ptr;
  R.nP0 = ar.get<double>((size_t)kPStride * ne);
  R.nP1 = ar.get<double>((size_t)kPStride * ne);
  R.nm = ar.get<double>(3 * ne);
  R.nv = ar.get<double>(3 * ne);
  R.nxo = ar.get<float>(3 * ne);
  R.nhot = ar.get<uint32_t>(ne);
  R.ne_list = ar.get<uint32_t>(ne);
  R.nlen = ar.get<uint32_t>(ne);
  R.wl = b.wl;
  k_permute_rows<<<nb, 256, 0, s>>>(R, ne);
  uint32_t *nrow_ptr = ar.get<uint32_t>(ne + 1);
  scan_u32_u32(R.nlen, nrow_ptr, ne, nrow_ptr + ne, ar, s);
  uint32_t *ncol = ar.get<uint32_t>(b.ninc ? b.ninc : 1);
  k_permute_cols<<<nb, 256, 0, s>>>(new_id, b.row_ptr, b.col, nrow_ptr, ne, ncol);
  k_hot_counts<<<(b.njobs + 255) / 256, 256, 0, s>>>(pos, total, nrow_ptr, b.e_off, b.njobs, ne,
                                                      b.wl_n, b.wl_step, b.wl_id, b.inc_n,
                                                      b.inc_step);
  b.P0 = R.nP0;
  b.P1 = R.nP1;
  b.m = R.nm;
  b.v = R.nv;
  b.xo = R.nxo;
  b.hot = R.nhot;
  b.row_ptr = nrow_ptr;
  b.col = ncol;
  e_list = R.ne_list;
}

// one wave per job: sums (and clears) the job's partial counts, sums its
// loss slots in slot order, then decides
__global__ void k_pgd_finalize(const PgdGroups *__restrict__ G) {
  const int ngroups = G->ngroups, lane = threadIdx.x;
  if ((int)blockIdx.x >= G->job_base[ngroups]) return;
  const int grp = ngroups > 1 ? group_of(G->job_base, ngroups, (int64_t)blockIdx.x) : 0;
  const PgdBufs &B = G->g[grp];
  const int j = (int)blockIdx.x - G->job_base[grp];
  JobLoop &L = B.loop[j];
  if (L.done) return;
  const JobDev &J = B.jobs[j];
  unsigned long long viol = 0;
  unsigned long long *a = B.acc + (size_t)j * B.acc_slots * 16;
  for (int k = lane; k < B.acc_slots; k += kWave) {
    viol += a[16 * k];
    a[16 * k] = 0;
  }
  viol = wsum(viol);
  // the slots written by this step: one per wave that walked a tile of the
  // job, i.e. of the first ceil(wl_step / 64) tiles
  const uint32_t wl = B.wl_step[j];
  const int64_t nslot = B.lp_off[j + 1] - B.lp_off[j];
  const int64_t used = (int64_t)(wl + 63u) / 64 < nslot ? (int64_t)(wl + 63u) / 64 : nslot;
  double loss = 0.0;
  for (int64_t k = lane; k < used; k += kWave) loss += B.lossp[B.lp_off[j] + k];
  loss = wsum_d(loss);
  if (lane != 0) return;
  L.rows_eval += wl;
  L.inc_eval += B.inc_step[j];
  if (!L.have0) {
    L.viol0 = viol;
    L.loss0 = loss;
    L.have0 = 1;
  }
  L.viol_last = viol;
  L.loss_last = loss;
  if (L.t < J.trace_cap) {
    J.trace_loss[L.t] = loss;
    J.trace_viol[L.t] = viol;
  }
  // Alg. 1's stopping test: no violated constraint, or the loss of Eq. 3 at
  // most eps_L when that is set
  const bool conv = J.loss_tol > 0.0 ? (loss <= J.loss_tol) : (viol == 0);
  if (conv || L.t >= J.max_iters) {
    L.done = 1;
    L.status = conv ? 0 : 1;
    atomicSub(B.n_active, 1);
    return;
  }
  // rows that became hot in this step join the next one (the worklist of
  // the first step is replaced by the compaction that follows it)
  if (L.t > 0) {
    B.wl_step[j] = B.wl_n[j];
    B.inc_step[j] = B.inc_n[j];
  }
  L.t += 1;
  const int64_t tb = L.t + 1 < J.bc_len ? L.t + 1 : J.bc_len - 1;
  L.bc1 = J.bc_tab[tb].x;
  L.bc2 = J.bc_tab[tb].y;
}

void launch_pgd_step(const PgdGroups *g, const PgdBufs &b, hipStream_t s) {
  if (b.ne) {
    // the loss slots were sized for this many waves
    if (b.nwaves != pgd_step_waves(b.ne)) throw Error(-3, "PGD step grid differs from its loss slots");
    // one call: the kernel with the buffers as its argument (the shared
    // loop launches the kernel over the group table instead)
    (void)g;
    k_pgd_rows<<<b.nwaves / kPgdWaves, 64 * kPgdWaves, 0, s>>>(b);
  }
}
void launch_pgd_finalize(const PgdGroups *g, const PgdBufs &b, hipStream_t s) {
  if (b.njobs) k_pgd_finalize<<<b.njobs, kWave, 0, s>>>(g);
}
void launch_pgd_step_shared(const PgdGroups *g, hipStream_t s) {
  k_pgd_step<<<kPgdBlocks, 64 * kPgdWaves, 0, s>>>(g);
}
void launch_pgd_finalize_shared(const PgdGroups *g, hipStream_t s) {
  k_pgd_finalize<<<kMaxGroupJobs, kWave, 0, s>>>(g);
}

}  // namespace pcc
