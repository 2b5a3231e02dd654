// Fixed-radius pair enumeration over the forward half shell of each cell
// (Sec. 2.4.1, Sec. 3.3), pair classes (Sec. 3.1, 3.2), lock-free union-find
// with minimum-index roots (Sec. 2.4.1), canonical labels, the mode filters of
// Sec. 3.2 and the halo-forest spanning forest by Boruvka rounds.
//
// Each sorted particle k is one thread; it compares itself with the later
// particles of its own cell and with every particle of the 13 forward
// neighbour cells, so every unordered pair within the search radius is seen
// exactly once.  A float32 test with a margin rejects far candidates; every
// candidate that passes is classified by the exact float64 squared distance
// (x, then y, then z, no contraction), the predicate the oracle evaluates.
#include "kernels.hpp"

#include <algorithm>
#include <cstdio>
#include <cstdlib>

namespace pcc {

enum : int { kNone = 0, kSafe = 1, kPb = 2, kPc = 3 };

// ----------------------------------------------------------------------------
// union-find on uint32 parents; roots are the smallest index of their set
// ----------------------------------------------------------------------------
__device__ inline uint32_t ld_par(const uint32_t *p, uint32_t i) {
  return __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_par(uint32_t *p, uint32_t i, uint32_t v) {
  __hip_atomic_store(p + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Find with path halving.  Parent reads are plain loads: a value read from a
// stale cache line is still an ancestor (parents only ever move to ancestors),
// and a stale "root" is caught by the compare-and-swap of the union, whose
// returned value lets the search go on from fresh data.
__device__ inline uint32_t uf_find(uint32_t *par, uint32_t x) {
  for (;;) {
    const uint32_t p = par[x];
    if (p == x) return x;
    const uint32_t gp = par[p];
    if (gp == p) return p;
    st_par(par, x, gp);
    x = gp;
  }
}

// Hook the larger root under the smaller one with a compare-and-swap.  On
// failure the swap returns the node's current parent, a strictly smaller
// index, and the search continues from there; so every retry makes progress.
// Returns the root the two sets now share (as far as this thread knows).
__device__ inline uint32_t uf_union(uint32_t *par, uint32_t a, uint32_t b) {
  a = uf_find(par, a);
  b = uf_find(par, b);
  for (;;) {
    if (a == b) return a;
    if (a < b) {
      const uint32_t t = a;
      a = b;
      b = t;
    }
    uint32_t seen = a;
    if (__hip_atomic_compare_exchange_strong(par + a, &seen, b, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return b;
    a = uf_find(par, seen);
    b = uf_find(par, b);
  }
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ----------------------------------------------------------------------------
// wave-aggregated per-job counters
// ----------------------------------------------------------------------------
__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Adds the counts of a wave's lanes to their jobs' counters.  Each job has
// `slots` copies of its K counters, each copy on its own 128-byte line; a
// wave adds into the copy of its index, so that no address takes more than
// a few atomics (same-address device atomics serialise).
template <int K>
__device__ inline void job_add(unsigned long long *ctr, int slots, int job, bool valid,
                               const unsigned long long (&v)[K]) {
  static_assert(K <= 16, "counters of one slot share a 128-byte line");
  const int jv = valid ? job : -1;
  uint64_t todo = __ballot(valid);
  const int lane = threadIdx.x & 63;
  const int slot = (int)(((size_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) &
                         (size_t)(slots - 1));
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int lj = __shfl(jv, leader, kWave);
    const uint64_t grp = __ballot(jv == lj);
#pragma unroll
    for (int c = 0; c < K; ++c) {
      const unsigned long long s = wave_sum_u64(jv == lj ? v[c] : 0ull);
      if (lane == leader && s) atomicAdd(ctr + ((size_t)lj * slots + slot) * 16 + c, s);
    }
    todo &= ~grp;
  }
}

// ----------------------------------------------------------------------------
// the pair kernel
// ----------------------------------------------------------------------------
struct JobPair {
  double rs2, b2, rv2, bm2;
  double L[3], hL[3];
  float Lf[3], hLf[3];
  float f_rs_lo, f_rs_hi, f_b_lo, f_b_hi, f_rv_lo, f_rv_hi;
  int mode;
  int img;
};

__device__ inline JobPair load_job(const JobDev &J) {
  JobPair q;
  q.rs2 = J.rs2;
  q.b2 = J.b2;
  q.rv2 = J.rv2;
  q.bm2 = J.bm2;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    q.L[a] = J.L[a];
    q.hL[a] = J.hL[a];
    q.Lf[a] = J.Lf[a];
    q.hLf[a] = J.hLf[a];
  }
  q.f_rs_lo = J.f_rs_lo;
  q.f_rs_hi = J.f_rs_hi;
  q.f_b_lo = J.f_b_lo;
  q.f_b_hi = J.f_b_hi;
  q.f_rv_lo = J.f_rv_lo;
  q.f_rv_hi = J.rv2_f32;
  q.mode = J.mode;
  q.img = J.img;
  return q;
}

__device__ inline float wrap_f(float d, float L, float hL) {
  if (d > hL)
    d -= L;
  else if (d < -hL)
    d += L;
  return d;
}
__device__ inline double wrap_d(double d, double L, double hL) {
  if (d > hL)
    d -= L;
  else if (d < -hL)
    d += L;
  return d;
}

// exact squared distance of the oracle: (dx*dx + dy*dy) + dz*dz in float64
__device__ inline double dist2_exact(const float4 &a, const float4 &b, const JobPair &q) {
  const double dx = wrap_d((double)a.x - (double)b.x, q.L[0], q.hL[0]);
  const double dy = wrap_d((double)a.y - (double)b.y, q.L[1], q.hL[1]);
  const double dz = wrap_d((double)a.z - (double)b.z, q.L[2], q.hL[2]);
  return (dx * dx + dy * dy) + dz * dz;
}

__device__ inline float axis_shift(int d, uint32_t edge, int a, float L) {
  if (d > 0 && ((edge >> (2 * a + 1)) & 1u)) return L;  // home on the high edge
  if (d < 0 && ((edge >> (2 * a)) & 1u)) return -L;     // home on the low edge
  return 0.f;
}
// Periodic image of neighbour slot `slot` (the neighbour table's order: the
// cell x + 1; then for the rows (dy, dz) = (1, 0), (-1, 1), (0, 1), (1, 1)
// the cells x - 1 .. x + 1 inside [0, nx) and the one across the x face) of
// a cell with face bits `edge`: a partner's displacement is (home - partner)
// - shift on every axis.  Zero unless the job's coordinates lie in its
// periodic box (the face bits are then clear and each candidate is wrapped
// instead).
__device__ inline float3 image_shift(int slot, uint32_t edge, const JobPair &q) {
  float sx;
  int dy = 0, dz = 0;
  if (slot == 0) {
    sx = axis_shift(1, edge, 0, q.Lf[0]);
  } else {
    const int g = (slot - 1) >> 1;
    dy = g == 0 ? 1 : (g == 1 ? -1 : (g == 2 ? 0 : 1));
    dz = g == 0 ? 0 : 1;
    // the cell across the x face: home on the low face (partner near L) or
    // on the high face (partner near 0)
    sx = (slot & 1) ? 0.f : ((edge & 1u) ? -q.Lf[0] : ((edge & 2u) ? q.Lf[0] : 0.f));
  }
  return make_float3(sx, axis_shift(dy, edge, 1, q.Lf[1]), axis_shift(dz, edge, 2, q.Lf[2]));
}

// Class of a candidate pair: a float32 squared distance decides whenever it
// lies outside the guard band of every threshold; inside a band, the exact
// float64 squared distance of the oracle decides.
__device__ inline int classify(const JobPair &q, const float4 &pi, const float4 &pj,
                               const float3 &sh) {
  float dx = (pi.x - pj.x) - sh.x;
  float dy = (pi.y - pj.y) - sh.y;
  float dz = (pi.z - pj.z) - sh.z;
  if (!q.img) {
    dx = wrap_f(dx, q.Lf[0], q.hLf[0]);
    dy = wrap_f(dy, q.Lf[1], q.hLf[1]);
    dz = wrap_f(dz, q.Lf[2], q.hLf[2]);
  }
  const float d2f = (dx * dx + dy * dy) + dz * dz;
  if (d2f > q.f_rv_hi) return kNone;
  if (d2f < q.f_rs_lo) return kSafe;
  if (d2f > q.f_rs_hi && d2f < q.f_b_lo) return kPb;
  if (d2f > q.f_b_hi && d2f < q.f_rv_lo) return kPc;
  const double d2 = dist2_exact(pi, pj, q);
  if (d2 > q.rv2) return kNone;
  return d2 <= q.rs2 ? kSafe : (d2 <= q.b2 ? kPb : kPc);
}

// Float32 squared distance from a home to a partner staged with the image
// shift of its range already added (ps = pj + shift, rounded once per
// staged partner): per axis pi - ps, again two roundings, and the squares
// summed with fused multiply-adds.  Its error stays inside the bound of the
// guard bands (one and a half float32 ulps per axis of max|x| + L + 1).
__device__ inline float dist2_staged(const JobPair &q, const float4 &pi, const float4 &ps) {
  float dx = pi.x - ps.x, dy = pi.y - ps.y, dz = pi.z - ps.z;
  if (!q.img) {
    dx = wrap_f(dx, q.Lf[0], q.hLf[0]);
    dy = wrap_f(dy, q.Lf[1], q.hLf[1]);
    dz = wrap_f(dz, q.Lf[2], q.hLf[2]);
  }
  return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}
// class from such a distance; inside a band the exact predicate decides on
// the partner's unshifted position
__device__ inline int class_staged(const JobPair &q, float d2f, const float4 &pi,
                                   const float4 *pos, uint32_t j) {
  if (d2f > q.f_rv_hi) return kNone;
  if (d2f < q.f_rs_lo) return kSafe;
  if (d2f > q.f_rs_hi && d2f < q.f_b_lo) return kPb;
  if (d2f > q.f_b_hi && d2f < q.f_rv_lo) return kPc;
  const double d2 = dist2_exact(pi, pos[j], q);
  if (d2 > q.rv2) return kNone;
  return d2 <= q.rs2 ? kSafe : (d2 <= q.b2 ? kPb : kPc);
}

// Box of a wave's home positions, and the test that drops a staged partner
// no home of the box can reach.  Per axis the partner's float32 gap to the
// box, fl(lo - ps) or fl(ps - hi), is at most |fl(h - ps)| for every home h
// in the box (rounding is monotonic), and the fused sum of squares is
// monotonic in each term, so a gap-distance above the r_v band's upper edge
// means every home's dist2_staged lies above it too, i.e. every exact
// distance exceeds r_v.  Only for jobs whose candidates are not wrapped.
struct HomeBox {
  float lo[3], hi[3];
};
__device__ inline HomeBox home_box(const float4 &pi, bool valid) {
  const float inf = __builtin_huge_valf();
  HomeBox b;
  b.lo[0] = valid ? pi.x : inf;
  b.lo[1] = valid ? pi.y : inf;
  b.lo[2] = valid ? pi.z : inf;
  b.hi[0] = valid ? pi.x : -inf;
  b.hi[1] = valid ? pi.y : -inf;
  b.hi[2] = valid ? pi.z : -inf;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      b.lo[a] = fminf(b.lo[a], __shfl_xor(b.lo[a], d, kWave));
      b.hi[a] = fmaxf(b.hi[a], __shfl_xor(b.hi[a], d, kWave));
    }
  return b;
}
__device__ inline bool box_reaches(const JobPair &q, const HomeBox &b, const float4 &ps) {
  const float ex = fmaxf(fmaxf(b.lo[0] - ps.x, ps.x - b.hi[0]), 0.f);
  const float ey = fmaxf(fmaxf(b.lo[1] - ps.y, ps.y - b.hi[1]), 0.f);
  const float ez = fmaxf(fmaxf(b.lo[2] - ps.z, ps.z - b.hi[2]), 0.f);
  return __builtin_fmaf(ez, ez, __builtin_fmaf(ey, ey, ex * ex)) <= q.f_rv_hi;
}

// State of one home particle k during a pass.
struct Home {
  uint32_t k;
  float4 pi, ri;
  uint32_t sk, fk;     // safe and FoF roots (passes 2 and 3); root guesses (pass 1)
  uint64_t wa, wf;     // write cursors (pass 3)
  uint32_t ca, cf;     // counts: pass 1 pc and pb pairs, pass 2 active and forest pairs
  uint32_t cs;         // pass 1: safe pairs
};

template <int PASS>
__device__ inline void home_begin(const PairBufs &B, Home &h, uint32_t k) {
  h.k = k;
  h.pi = B.pos[k];
  h.ri = make_float4(0.f, 0.f, 0.f, 0.f);
  h.sk = h.fk = k;
  if (PASS >= 2) {
    h.sk = B.safe_par[k];
    h.fk = B.fof_par[k];
  }
  if (PASS == 3) h.ri = B.rec[k];
  h.wa = PASS == 3 ? B.off_a[k] : 0;
  h.wf = PASS == 3 ? B.off_f[k] : 0;
  h.ca = h.cf = h.cs = 0;
}

template <int PASS>
__device__ inline void home_end(const PairBufs &B, const Home &h) {
  if (PASS == 1) {
    B.cnt_pb[h.k] = h.cf;  // potentially broken (safe < d <= b)
    B.cnt_pc[h.k] = h.ca;  // potentially created (b < d <= r_v)
  }
  if (PASS == 2) {
    B.cnt_a[h.k] = h.ca;
    B.cnt_f[h.k] = h.cf;
  }
  if (PASS == 3 && B.slotted) {
    // slots sized by pass 1's class counts: record the fill of the active
    // slots; unused forest slots become self-loops of the home's safe
    // component, which the spanning forest ignores
    B.cnt_a[h.k] = (uint32_t)(h.wa - B.off_a[h.k]);
    const uint64_t fend = B.off_f[h.k] + B.cap_f[h.k];
    for (uint64_t w = h.wf; w < fend; ++w) {
      B.f_key[w] = ~0ull;
      B.f_u[w] = h.sk;
      B.f_v[w] = h.sk;
    }
  }
}

// Mode filter of a vulnerable pair (Sec. 3.2): to_a for the active list,
// to_f for the halo forest's candidates.  spj / fpj: the partner's safe and
// FoF roots.
__device__ inline void mode_filter(const JobPair &q, const Home &h, int cls, uint32_t spj,
                                   uint32_t fpj, bool &to_a, bool &to_f) {
  to_a = to_f = false;
  if (cls == kNone || cls == kSafe) return;
  if (q.mode == 0)
    to_a = true;
  else if (q.mode == 1)
    to_a = spj != h.sk;
  else if (cls == kPc)
    to_a = fpj != h.fk;
  else
    to_f = spj != h.sk;
}

// Forest key of a candidate: links already broken in the reconstruction
// last, then the pair of job-local indices.
__device__ inline uint64_t forest_key(const PairBufs &B, const JobPair &q, const Home &h, uint32_t j,
                                      const float4 &pj) {
  const float4 rj = B.rec[j];
  const double ex = wrap_d((double)h.ri.x - (double)rj.x, q.L[0], q.hL[0]);
  const double ey = wrap_d((double)h.ri.y - (double)rj.y, q.L[1], q.hL[1]);
  const double ez = wrap_d((double)h.ri.z - (double)rj.z, q.L[2], q.hL[2]);
  const uint64_t viol0 = ((ex * ex + ey * ey) + ez * ez) > q.bm2 ? 1ull : 0ull;
  const uint32_t li = __float_as_uint(h.pi.w), lj = __float_as_uint(pj.w);
  const uint64_t lo = li < lj ? li : lj, hi = li < lj ? lj : li;
  return (viol0 << 62) | (lo << 31) | hi;
}

// The same key from the home's reconstructed position and job-local index
// (the write pass's queued candidates carry the home's lane, not its state).
__device__ inline uint64_t forest_key_of(const PairBufs &B, const JobPair &q, const float4 &ri,
                                         uint32_t li, uint32_t j, uint32_t lj) {
  const float4 rj = B.rec[j];
  const double ex = wrap_d((double)ri.x - (double)rj.x, q.L[0], q.hL[0]);
  const double ey = wrap_d((double)ri.y - (double)rj.y, q.L[1], q.hL[1]);
  const double ez = wrap_d((double)ri.z - (double)rj.z, q.L[2], q.hL[2]);
  const uint64_t viol0 = ((ex * ex + ey * ey) + ez * ez) > q.bm2 ? 1ull : 0ull;
  const uint64_t lo = li < lj ? li : lj, hi = li < lj ? lj : li;
  return (viol0 << 62) | (lo << 31) | hi;
}

// One candidate partner j of the home particle: its class, then the work of
// the pass.  STAGED says which of the partner's parents come from the caller
// (bit 0 the safe parent, bit 1 the FoF parent: staged or loaded ahead with
// its position); the others are read when needed.  In pass 1 a parent
// only serves to skip a union that is already done: a node's parent only
// ever moves to an ancestor, so a stale value equal to the home's root guess
// still means both are in one set, and any other value leads to a union.
template <int PASS, int STAGED>
__device__ inline void visit_class(const PairBufs &B, const JobPair &q, Home &h, uint32_t j,
                                   const float4 &pj, int cls, uint32_t sj, uint32_t fj) {
  if (cls == kNone) return;
  auto spar = [&]() { return (STAGED & 1) ? sj : B.safe_par[j]; };
  auto fpar = [&]() { return (STAGED & 2) ? fj : B.fof_par[j]; };
  if (PASS == 1) {
    // h.sk / h.fk hold an ancestor of k in each forest: a partner whose
    // parent is that node is already in k's set and needs no union
    if (cls == kSafe) {
      h.cs++;
      if (spar() != h.sk) h.sk = uf_union(B.safe_par, h.sk, j);
      if (fpar() != h.fk) h.fk = uf_union(B.fof_par, h.fk, j);
    } else if (cls == kPb) {
      h.cf++;
      if (fpar() != h.fk) h.fk = uf_union(B.fof_par, h.fk, j);
    } else {
      h.ca++;
    }
    return;
  }
  if (cls == kSafe) return;
  bool to_a, to_f;
  const uint32_t spj = (q.mode == 0 || (q.mode == 2 && cls == kPc)) ? 0u : spar();
  const uint32_t fpj = (q.mode == 2 && cls == kPc) ? fpar() : 0u;
  mode_filter(q, h, cls, spj, fpj, to_a, to_f);
  if (PASS == 2) {
    h.ca += to_a;
    h.cf += to_f;
    return;
  }
  if (to_a) {
    B.a_i[h.wa] = h.k;
    B.a_j[h.wa] = j;
    B.a_t[h.wa] = (uint8_t)cls;
    h.wa++;
  }
  if (to_f) {
    B.f_key[h.wf] = forest_key(B, q, h, j, pj);
    B.f_u[h.wf] = h.sk;
    B.f_v[h.wf] = spj;
    h.wf++;
  }
}

template <int PASS, int STAGED>
__device__ inline void visit(const PairBufs &B, const JobPair &q, Home &h, uint32_t j,
                             const float4 &pj, const float3 &sh, uint32_t sj, uint32_t fj) {
  visit_class<PASS, STAGED>(B, q, h, j, pj, classify(q, h.pi, pj, sh), sj, fj);
}

__device__ inline void pass1_counts(const Home &h, bool valid, unsigned long long (&cnt)[3]) {
  cnt[0] = valid ? h.cs : 0u;
  cnt[1] = valid ? h.cf : 0u;
  cnt[2] = valid ? h.ca : 0u;
}

// Sparse cells: one thread per particle (list of particles of cells below
// the dense-cell threshold, ordered by the candidate count of their cell).
// Partners: later particles of its own cell, then the particles of the 13
// forward cells, which the neighbour table gives as kNbrSlots ranges of the
// sorted order (runs of cells with consecutive keys).  The ranges are read
// at once (one contiguous row of the table) and kept in LDS; the walk over
// them is one flat loop, one candidate per lane per iteration, so a lane
// stays busy until its own candidates run out (nested loops over the
// ranges would idle every lane whose current range is shorter than the
// longest one in the wave); the next candidate's position is loaded before
// the current one is examined.
constexpr int kSparseThreads = 256;
constexpr int kRanges = 1 + kNbrSlots;  // the home cell, then the neighbour slots

template <int PASS>
__global__ void __launch_bounds__(kSparseThreads) k_pairs_sparse(PairBufs B, const uint32_t *list,
                                                                 size_t m) {
  // candidate ranges [lo, hi) of each thread: range 0 the home cell, range
  // r > 0 neighbour slot r - 1; [range][thread], so a wave's accesses to one
  // range fall in distinct banks
  __shared__ uint32_t r_lo[kRanges][kSparseThreads], r_hi[kRanges][kSparseThreads];
  unsigned long long cnt[3] = {0ull, 0ull, 0ull};  // safe, pb, pc
  const int tid = threadIdx.x;
  const size_t t = (size_t)blockIdx.x * blockDim.x + tid;
  const int cjob = t < m ? job_of(B.p_off, B.njobs, (int64_t)list[t]) : -1;
  if (t < m) {
    const uint32_t k = list[t];
    const JobPair q = load_job(B.jobs[cjob]);
    Home h;
    home_begin<PASS>(B, h, k);
    const uint32_t cell = B.cell_of[k];
    const uint2 *nr_row = B.nrange + (size_t)cell * kNbrSlots;
    const uint32_t edge = B.cell_edge[cell];
    r_lo[0][tid] = k + 1;
    r_hi[0][tid] = B.cell_start[cell + 1];
#pragma unroll
    for (int i = 0; i < kNbrSlots; ++i) {
      const uint2 v = nr_row[i];
      r_lo[i + 1][tid] = v.x;
      r_hi[i + 1][tid] = v.y;
    }
    auto enter = [&](int r, uint32_t &j, uint32_t &e, float3 &sh) {
      j = r_lo[r][tid];
      e = r_hi[r][tid];
      sh = r == 0 ? make_float3(0.f, 0.f, 0.f) : image_shift(r - 1, edge, q);
    };
    // (j, e): the current range r; empty ranges are passed over
    int r = 0;
    uint32_t j = 0, e = 0;
    float3 sh = make_float3(0.f, 0.f, 0.f);
    enter(0, j, e, sh);
    while (j >= e && ++r < kRanges) enter(r, j, e, sh);
    // the partner's position and parents are loaded one candidate ahead (the
    // FoF parent in pass 1, where the safe one is rarely needed; both after)
    constexpr int kAhead = PASS == 1 ? 2 : 3;
    uint32_t ja = r < kRanges ? j : k;  // (index k: any valid load)
    float4 pj = B.pos[ja];
    uint32_t sj = (kAhead & 1) ? B.safe_par[ja] : 0u, fj = B.fof_par[ja];
    while (r < kRanges) {
      uint32_t jn = j + 1, en = e;
      int rn = r;
      float3 shn = sh;
      while (jn >= en && ++rn < kRanges) enter(rn, jn, en, shn);
      ja = rn < kRanges ? jn : k;
      const float4 pn = B.pos[ja];
      const uint32_t sn = (kAhead & 1) ? B.safe_par[ja] : 0u, fn = B.fof_par[ja];
      visit<PASS, kAhead>(B, q, h, j, pj, sh, sj, fj);
      j = jn;
      e = en;
      r = rn;
      sh = shn;
      pj = pn;
      sj = sn;
      fj = fn;
    }
    home_end<PASS>(B, h);
    if (PASS == 1) pass1_counts(h, true, cnt);
  }
  if (PASS == 1) job_add<3>(B.job_counts, B.count_slots, cjob, cjob >= 0, cnt);
}

constexpr int kPairWaves = 4;

// Stages the partners t0 .. t0 + cnt - 1 of a dense unit in LDS, each lane
// loading one: its position with the range's image shift added, both
// parents and its index.  With `cull` (a neighbour range of a job whose
// candidates are not wrapped), a partner that no home of the unit's box
// can reach is left out; the others keep their order.  Returns how many
// were staged.
__device__ inline uint32_t stage_partners(const PairBufs &B, const JobPair &q, const HomeBox &box,
                                          bool cull, uint32_t t0, uint32_t cnt, const float3 &sh,
                                          int lane, uint64_t below, float4 *stage, uint32_t *ssp,
                                          uint32_t *sfp, uint32_t *sidx) {
  bool keep = false;
  float4 ps = make_float4(0.f, 0.f, 0.f, 0.f);
  if ((uint32_t)lane < cnt) {
    const float4 p = B.pos[t0 + lane];
    ps = make_float4(p.x + sh.x, p.y + sh.y, p.z + sh.z, p.w);
    keep = !(cull && q.img) || box_reaches(q, box, ps);
  }
  const uint64_t km = __ballot(keep);
  if (keep) {
    const uint32_t d = (uint32_t)__popcll(km & below);
    stage[d] = ps;
    ssp[d] = B.safe_par[t0 + lane];
    sfp[d] = B.fof_par[t0 + lane];
    sidx[d] = t0 + lane;
  }
  wave_sync();
  return (uint32_t)__popcll(km);
}

// Dense cells: one wave per 64 home particles of one cell.  Each neighbour
// range (a run of forward cells with consecutive keys) is staged through
// LDS 64 particles at a time with coalesced loads (positions and both
// parents); every lane then runs over the same staged particles (broadcast
// reads), so the lanes of a wave never diverge on trip counts, and the
// periodic image of a range is one shift for the whole wave.  Every home
// particle sees its partners in the same order as in the sparse kernel.
template <int PASS>
__global__ void __launch_bounds__(64 * kPairWaves) k_pairs_dense(PairBufs B, const uint32_t *ucell,
                                                                 const uint32_t *uchunk, size_t m) {
  __shared__ float4 stage[kPairWaves][64];
  __shared__ uint32_t ssp[kPairWaves][64], sfp[kPairWaves][64], sidx[kPairWaves][64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const size_t unit = (size_t)blockIdx.x * kPairWaves + w;
  if (unit >= m) return;  // the whole wave leaves together
  const uint32_t cell = ucell[unit];
  const uint32_t cs = B.cell_start[cell], ce = B.cell_start[cell + 1];
  const uint32_t k0 = cs + 64u * uchunk[unit];
  const uint32_t nh = (ce - k0) < 64u ? (ce - k0) : 64u;
  const bool valid = (uint32_t)lane < nh;
  const int job = __builtin_amdgcn_readfirstlane(job_of(B.p_off, B.njobs, (int64_t)k0));
  const JobPair q = load_job(B.jobs[job]);
  const uint32_t edge = B.cell_edge[cell];
  Home h;
  home_begin<PASS>(B, h, valid ? k0 + lane : k0);
  const HomeBox box = home_box(h.pi, valid);
  const uint64_t below = (1ull << lane) - 1ull;
  for (int s = 0; s <= kNbrSlots; ++s) {
    uint32_t j0, j1;
    float3 sh = make_float3(0.f, 0.f, 0.f);
    if (s == 0) {
      j0 = k0 + 1;  // later particles of the home cell
      j1 = ce;
    } else {
      const uint2 v = B.nrange[(size_t)cell * kNbrSlots + s - 1];
      if (v.x >= v.y) continue;
      j0 = v.x;
      j1 = v.y;
      sh = image_shift(s - 1, edge, q);
    }
    for (uint32_t t0 = j0; t0 < j1; t0 += 64) {
      const uint32_t cnt_t = (j1 - t0) < 64u ? (j1 - t0) : 64u;
      const uint32_t nk = stage_partners(B, q, box, s > 0, t0, cnt_t, sh, lane, below, stage[w],
                                         ssp[w], sfp[w], sidx[w]);
      if (valid) {
        auto one = [&](uint32_t t) {
          const float4 ps = stage[w][t];
          const uint32_t j = sidx[w][t];
          visit_class<PASS, 3>(B, q, h, j, ps,
                                  class_staged(q, dist2_staged(q, h.pi, ps), h.pi, B.pos, j),
                                  ssp[w][t], sfp[w][t]);
        };
        if (s == 0) {
          // the home cell is staged whole: only the partners after k
          for (uint32_t t = h.k >= t0 ? h.k + 1 - t0 : 0u; t < nk; ++t) one(t);
        } else {
          for (uint32_t t = 0; t < nk; ++t) one(t);
        }
      }
      wave_sync();
    }
  }
  if (valid) home_end<PASS>(B, h);
  if (PASS == 1) {
    unsigned long long cnt[3];
    pass1_counts(h, valid, cnt);
    job_add<3>(B.job_counts, B.count_slots, job, valid, cnt);
  }
}

// Write pass over dense cells.  The 64 home particles of a unit are
// consecutive, so their slots form one block; the kept pairs are appended
// to that block at a wave-wide cursor (ballot and prefix count), in the
// order (partner, home lane), which turns the stores into contiguous runs.
// The first home of the unit records the block's fill; unused forest slots
// at the block's end become self-loops.
__global__ void __launch_bounds__(64 * kPairWaves) k_pairs_dense_write(PairBufs B,
                                                                       const uint32_t *ucell,
                                                                       const uint32_t *uchunk,
                                                                       size_t m) {
  __shared__ float4 stage[kPairWaves][64];
  __shared__ uint32_t ssp[kPairWaves][64], sfp[kPairWaves][64], sidx[kPairWaves][64];
  // forest candidates wait in a queue (home lane | staged index << 6, in
  // the order partner, home lane) and are keyed and stored 64 at a time with
  // every lane busy, instead of by the few lanes that find one per partner
  __shared__ uint16_t fq[kPairWaves][128];
  __shared__ float4 hri[kPairWaves][64];  // the homes' reconstructed positions
  __shared__ uint32_t hsk[kPairWaves][64], hli[kPairWaves][64];  // safe roots, local ids
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const size_t unit = (size_t)blockIdx.x * kPairWaves + w;
  if (unit >= m) return;  // the whole wave leaves together
  const uint32_t cell = ucell[unit];
  const uint32_t cs = B.cell_start[cell], ce = B.cell_start[cell + 1];
  const uint32_t k0 = cs + 64u * uchunk[unit];
  const uint32_t nh = (ce - k0) < 64u ? (ce - k0) : 64u;
  const bool valid = (uint32_t)lane < nh;
  const int job = __builtin_amdgcn_readfirstlane(job_of(B.p_off, B.njobs, (int64_t)k0));
  const JobPair q = load_job(B.jobs[job]);
  const uint32_t edge = B.cell_edge[cell];
  Home h;
  home_begin<3>(B, h, valid ? k0 + lane : k0);
  const HomeBox box = home_box(h.pi, valid);
  const uint64_t a0 = B.off_a[k0], f0 = B.off_f[k0];
  uint64_t wa = a0, wf = f0;
  const uint64_t below = (1ull << lane) - 1ull;
  hri[w][lane] = h.ri;
  hsk[w][lane] = h.sk;
  hli[w][lane] = __float_as_uint(h.pi.w);
  uint32_t qn = 0;  // queued forest candidates (wave-uniform)
  // keys and stores the first cnt (<= 64) queued candidates
  auto flush = [&](uint32_t cnt) {
    if ((uint32_t)lane < cnt) {
      const uint32_t e = fq[w][lane], hl = e & 63u, t = e >> 6;
      const uint32_t j = sidx[w][t];
      const uint64_t d = wf + (uint64_t)lane;
      B.f_key[d] = forest_key_of(B, q, hri[w][hl], hli[w][hl], j, __float_as_uint(stage[w][t].w));
      B.f_u[d] = hsk[w][hl];
      B.f_v[d] = ssp[w][t];
    }
    wf += cnt;
  };
  for (int s = 0; s <= kNbrSlots; ++s) {
    uint32_t j0, j1;
    float3 sh = make_float3(0.f, 0.f, 0.f);
    if (s == 0) {
      j0 = k0 + 1;  // later particles of the home cell
      j1 = ce;
    } else {
      const uint2 v = B.nrange[(size_t)cell * kNbrSlots + s - 1];
      if (v.x >= v.y) continue;
      j0 = v.x;
      j1 = v.y;
      sh = image_shift(s - 1, edge, q);
    }
    for (uint32_t t0 = j0; t0 < j1; t0 += 64) {
      const uint32_t cnt_t = (j1 - t0) < 64u ? (j1 - t0) : 64u;
      const uint32_t nk = stage_partners(B, q, box, s > 0, t0, cnt_t, sh, lane, below, stage[w],
                                         ssp[w], sfp[w], sidx[w]);
      for (uint32_t t = 0; t < nk; ++t) {
        const uint32_t j = sidx[w][t];
        const float4 pj = stage[w][t];
        int cls = kNone;
        bool ta = false, tf = false;
        if (valid && !(s == 0 && j <= h.k)) {
          cls = class_staged(q, dist2_staged(q, h.pi, pj), h.pi, B.pos, j);
          mode_filter(q, h, cls, ssp[w][t], sfp[w][t], ta, tf);
        }
        const uint64_t ba = __ballot(ta), bf = __ballot(tf);
        if (ta) {
          const uint64_t d = wa + (uint64_t)__popcll(ba & below);
          B.a_i[d] = h.k;
          B.a_j[d] = j;
          B.a_t[d] = (uint8_t)cls;
        }
        wa += (uint64_t)__popcll(ba);
        if (bf) {
          if (tf) fq[w][qn + (uint32_t)__popcll(bf & below)] = (uint16_t)((uint32_t)lane | (t << 6));
          qn += (uint32_t)__popcll(bf);
          if (qn >= 64) {
            wave_sync();
            flush(64);
            const uint32_t rest = qn - 64;  // below 64
            const uint16_t mv = (uint32_t)lane < rest ? fq[w][64 + lane] : (uint16_t)0;
            wave_sync();
            if ((uint32_t)lane < rest) fq[w][lane] = mv;
            qn = rest;
          }
        }
      }
      // the staged partners are replaced next: key the queue's rest now
      wave_sync();
      flush(qn);
      qn = 0;
      wave_sync();
    }
  }
  if (B.slotted) {
    if (valid) B.cnt_a[h.k] = lane == 0 ? (uint32_t)(wa - a0) : 0u;
    const uint32_t last = k0 + nh - 1;
    const uint64_t fend = B.off_f[last] + B.cap_f[last];
    for (uint64_t x = wf + lane; x < fend; x += 64) {
      B.f_key[x] = ~0ull;
      B.f_u[x] = k0;
      B.f_v[x] = k0;
    }
  }
}

// particles of sparse cells, and (cell, 64-chunk) units of dense cells
__global__ void k_sparse_flags(const uint32_t *cell_of, const uint32_t *cell_start, size_t n,
                               uint32_t dense, uint8_t *flag) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x) {
    const uint32_t c = cell_of[k];
    flag[k] = (cell_start[c + 1] - cell_start[c]) < dense ? 1 : 0;
  }
}
// list[pos32[k]] = src ? src[k] : k for every flagged k (order kept)
__global__ void k_sparse_list(const uint8_t *flag, const uint32_t *pos32, size_t n,
                              const uint32_t *src, uint32_t *list) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x)
    if (flag[k]) list[pos32[k]] = src ? src[k] : (uint32_t)k;
}
// Bucket of a sparse particle by the number of particles in its cell and its
// 13 forward cells (the candidates it examines), doubling ranges, heaviest
// first: the lanes of a wave then have similar trip counts, while within a
// bucket the particles keep their (spatial) order for cache reuse.
__global__ void k_sparse_keys(const uint32_t *list, size_t m, const uint32_t *cell_of,
                              const uint32_t *cell_start, const uint2 *nrange, uint32_t *key) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (size_t)gridDim.x * blockDim.x) {
    const uint32_t c = cell_of[list[i]];
    uint32_t cost = cell_start[c + 1] - cell_start[c];
    for (int s = 0; s < kNbrSlots; ++s) {
      const uint2 v = nrange[(size_t)c * kNbrSlots + s];
      cost += v.y - v.x;
    }
    const uint32_t lg = 31u - (uint32_t)__clz(cost | 1u);  // floor(log2), 0 for cost <= 1
    key[i] = 15u - (lg < 15u ? lg : 15u);
  }
}

__global__ void k_unit_counts(const uint32_t *cell_start, const uint32_t *n_cells, size_t max_cells,
                              uint32_t dense, uint32_t *units) {
  const uint32_t U = *n_cells;
  for (size_t u = (size_t)blockIdx.x * blockDim.x + threadIdx.x; u < max_cells;
       u += (size_t)gridDim.x * blockDim.x) {
    uint32_t c = 0;
    if (u < U) {
      const uint32_t nu = cell_start[u + 1] - cell_start[u];
      c = nu >= dense ? (nu + 63u) / 64u : 0u;
    }
    units[u] = c;
  }
}
__global__ void k_unit_list(const uint32_t *units, const uint32_t *uoff, size_t max_cells,
                            uint32_t *ucell, uint32_t *uchunk) {
  for (size_t u = (size_t)blockIdx.x * blockDim.x + threadIdx.x; u < max_cells;
       u += (size_t)gridDim.x * blockDim.x)
    for (uint32_t c = 0; c < units[u]; ++c) {
      ucell[uoff[u] + c] = (uint32_t)u;
      uchunk[uoff[u] + c] = c;
    }
}

void plan_pairs(PairPlan &pl, const uint32_t *cell_of, const uint32_t *cell_start,
                const uint2 *nrange, const uint32_t *n_cells, size_t n, uint32_t dense, Arena &ar,
                hipStream_t s) {
  if (dense < 1) dense = 1;
  uint8_t *flag = ar.get<uint8_t>(n ? n : 1);
  uint32_t *pos32 = ar.get<uint32_t>(n ? n : 1);
  uint32_t *cnt = ar.get<uint32_t>(2);
  pl.sparse = ar.get<uint32_t>(n ? n : 1);
  uint32_t *units = ar.get<uint32_t>(n ? n : 1), *uoff = ar.get<uint32_t>(n ? n : 1);
  pl.ucell = ar.get<uint32_t>(n ? n : 1);
  pl.uchunk = ar.get<uint32_t>(n ? n : 1);
  const int nb = blocks_for(n, 256, 65536);
  if (n) {
    k_sparse_flags<<<nb, 256, 0, s>>>(cell_of, cell_start, n, dense, flag);
    scan_u8_u32(flag, pos32, n, cnt, ar, s);
    k_sparse_list<<<nb, 256, 0, s>>>(flag, pos32, n, nullptr, pl.sparse);
    // heaviest cells first, a cell's particles together and in index order
    uint32_t ns = 0;
    PCC_HIP(hipMemcpyAsync(&ns, cnt, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    PCC_HIP(hipStreamSynchronize(s));
    if (ns > 1) {
      uint32_t *key = ar.get<uint32_t>(ns);
      k_sparse_keys<<<blocks_for(ns, 256, 65536), 256, 0, s>>>(pl.sparse, ns, cell_of, cell_start,
                                                               nrange, key);
      radix_sort_u32(key, pl.sparse, ns, 4, ar, s);
    }
    k_unit_counts<<<nb, 256, 0, s>>>(cell_start, n_cells, n, dense, units);
    scan_u32_u32(units, uoff, n, cnt + 1, ar, s);
    k_unit_list<<<nb, 256, 0, s>>>(units, uoff, n, pl.ucell, pl.uchunk);
  } else {
    fill_u32(cnt, 0, 2, s);
  }
  uint32_t h[2] = {0, 0};
  PCC_HIP(hipMemcpyAsync(h, cnt, sizeof h, hipMemcpyDeviceToHost, s));
  PCC_HIP(hipStreamSynchronize(s));
  pl.n_sparse = h[0];
  pl.n_units = h[1];
}

template <int PASS>
static void launch_pairs(const PairBufs &b, const PairPlan &pl, hipStream_t s) {
  if (pl.n_sparse)
    k_pairs_sparse<PASS><<<blocks_for(pl.n_sparse, kSparseThreads, 1 << 30), kSparseThreads, 0,
                           s>>>(b, pl.sparse, pl.n_sparse);
  if (pl.n_units) {
    const unsigned nb = (unsigned)((pl.n_units + kPairWaves - 1) / kPairWaves);
    if (PASS == 3)
      k_pairs_dense_write<<<nb, 64 * kPairWaves, 0, s>>>(b, pl.ucell, pl.uchunk, pl.n_units);
    else
      k_pairs_dense<PASS><<<nb, 64 * kPairWaves, 0, s>>>(b, pl.ucell, pl.uchunk, pl.n_units);
  }
}

// Sparse homes that found a vulnerable pair in pass 1 (the count and write
// passes see no other pairs, so a home without one writes nothing).
__global__ void k_vul_flags(const uint32_t *list, size_t m, const uint32_t *cnt_pb,
                            const uint32_t *cnt_pc, uint8_t *flag) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (size_t)gridDim.x * blockDim.x) {
    const uint32_t k = list[i];
    flag[i] = (cnt_pb[k] | cnt_pc[k]) != 0u ? 1 : 0;
  }
}

void plan_vulnerable(const PairPlan &pl, const uint32_t *cnt_pb, const uint32_t *cnt_pc,
                     PairPlan &out, Arena &ar, hipStream_t s) {
  out = pl;
  if (pl.n_sparse == 0) return;
  const size_t m = pl.n_sparse;
  uint8_t *flag = ar.get<uint8_t>(m);
  uint32_t *pos32 = ar.get<uint32_t>(m), *cnt = ar.get<uint32_t>(1);
  out.sparse = ar.get<uint32_t>(m);
  const int nb = blocks_for(m, 256, 65536);
  k_vul_flags<<<nb, 256, 0, s>>>(pl.sparse, m, cnt_pb, cnt_pc, flag);
  scan_u8_u32(flag, pos32, m, cnt, ar, s);
  k_sparse_list<<<nb, 256, 0, s>>>(flag, pos32, m, pl.sparse, out.sparse);
  uint32_t h = 0;
  PCC_HIP(hipMemcpyAsync(&h, cnt, sizeof h, hipMemcpyDeviceToHost, s));
  PCC_HIP(hipStreamSynchronize(s));
  out.n_sparse = h;
}

void launch_pair_pass1(const PairBufs &b, const PairPlan &pl, hipStream_t s) {
  launch_pairs<1>(b, pl, s);
}
void launch_pair_count(const PairBufs &b, const PairPlan &pl, hipStream_t s) {
  launch_pairs<2>(b, pl, s);
}
void launch_pair_write(const PairBufs &b, const PairPlan &pl, hipStream_t s) {
  launch_pairs<3>(b, pl, s);
}

__global__ void k_slot_caps(PairBufs B, uint32_t *cap_a, uint32_t *cap_f) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < B.n;
       k += (size_t)gridDim.x * blockDim.x) {
    const int j = job_of(B.p_off, B.njobs, (int64_t)k);
    const bool hf = B.jobs[j].mode == 2;
    cap_a[k] = hf ? B.cnt_pc[k] : B.cnt_pb[k] + B.cnt_pc[k];
    cap_f[k] = hf ? B.cnt_pb[k] : 0u;
  }
}

void pair_slot_caps(const PairBufs &b, uint32_t *cap_a, uint32_t *cap_f, hipStream_t s) {
  if (b.n) k_slot_caps<<<blocks_for(b.n, 256, 65536), 256, 0, s>>>(b, cap_a, cap_f);
}

__global__ void k_compact_slots(const uint32_t *a_i, const uint32_t *a_j, const uint8_t *a_t,
                                const uint64_t *off_slot, const uint32_t *fill,
                                const uint64_t *off_dense, size_t n, uint32_t *d_i,
                                uint32_t *d_j, uint8_t *d_t) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x) {
    const uint64_t s0 = off_slot[k], d0 = off_dense[k];
    for (uint32_t c = 0; c < fill[k]; ++c) {
      d_i[d0 + c] = a_i[s0 + c];
      d_j[d0 + c] = a_j[s0 + c];
      d_t[d0 + c] = a_t[s0 + c];
    }
  }
}

void compact_slots(const uint32_t *a_i, const uint32_t *a_j, const uint8_t *a_t,
                   const uint64_t *off_slot, const uint32_t *fill, const uint64_t *off_dense,
                   size_t n, uint32_t *d_i, uint32_t *d_j, uint8_t *d_t, hipStream_t s) {
  if (n)
    k_compact_slots<<<blocks_for(n, 256, 65536), 256, 0, s>>>(a_i, a_j, a_t, off_slot, fill,
                                                              off_dense, n, d_i, d_j, d_t);
}

// root of x without writing anything on the way
__device__ inline uint32_t uf_root_ro(const uint32_t *par, uint32_t x) {
  for (;;) {
    const uint32_t p = ld_par(par, x);
    if (p == x) return x;
    x = p;
  }
}

// After the hooks: every node points at its root.  Only the owner of a node
// writes it, and it writes the root, so concurrent walks see either an
// ancestor or the root and nothing can undo a finished entry (a halving
// store from another thread could, which is why finds here do not halve).
__global__ void k_flatten(uint32_t *par, size_t n) {
  for (size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
       x += (size_t)gridDim.x * blockDim.x)
    st_par(par, (uint32_t)x, uf_root_ro(par, (uint32_t)x));
}

void launch_flatten(uint32_t *par, size_t n, hipStream_t s) {
  if (n) k_flatten<<<blocks_for(n, 256, 65536), 256, 0, s>>>(par, n);
}

// canonical label: the smallest job-local index of the component
// Smallest job-local index per component.  Sorted neighbours mostly share
// their root, and many atomics on one address serialise: a segmented
// minimum over runs of lanes with equal roots leaves one atomic per run (the
// run's last lane), and a read of the current minimum skips atomics that
// cannot lower it.
__global__ void k_minid(const uint32_t *root, const float4 *pos, size_t n, uint32_t *minid) {
  const int lane = threadIdx.x & 63;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  // the loop runs the same number of times in every lane of a wave
  for (size_t base = (size_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < n;
       base += stride) {
    const size_t k = base + lane;
    const bool valid = k < n;
    const uint32_t r = valid ? root[k] : 0xffffffffu;
    uint32_t id = valid ? __float_as_uint(pos[k].w) : 0xffffffffu;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t r2 = __shfl_up(r, d, 64), id2 = __shfl_up(id, d, 64);
      if (lane >= d && r2 == r) id = id2 < id ? id2 : id;
    }
    const uint32_t rn = __shfl_down(r, 1, 64);
    const bool tail = valid && (lane == 63 || k + 1 >= n || rn != r);
    if (tail && id < minid[r]) atomicMin(minid + r, id);
  }
}
__global__ void k_labels(const uint32_t *root, const float4 *pos, const int64_t *p_off, int njobs,
                         size_t n, const uint32_t *minid, int32_t *lab) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x) {
    const int j = job_of(p_off, njobs, (int64_t)k);
    lab[p_off[j] + __float_as_uint(pos[k].w)] = (int32_t)minid[root[k]];
  }
}

void launch_labels(const uint32_t *root, const float4 *pos, const int64_t *p_off, int njobs,
                   size_t n, uint32_t *minid, int32_t *lab, hipStream_t s) {
  if (!n) return;
  fill_u32(minid, 0xffffffffu, n, s);
  const int nb = blocks_for(n, 256, 65536);
  k_minid<<<nb, 256, 0, s>>>(root, pos, n, minid);
  k_labels<<<nb, 256, 0, s>>>(root, pos, p_off, njobs, n, minid, lab);
}

// ----------------------------------------------------------------------------
// Boruvka rounds on the supernode multigraph (Sec. 3.2 halo-forest mode).
// With distinct keys the minimum spanning forest is unique, so this equals
// Kruskal's forest in ascending key order.
// ----------------------------------------------------------------------------
// At the start of a round every candidate holds the current roots of its two
// ends (safe roots in the first round, relabelled ones after), so no find is
// needed until the round's unions.  A candidate whose ends share a root is
// dead (the first round's unused slots are such self-loops).
//
// Each live edge offers its key to the best (smallest) edge of both of its
// components.  Edges of one home particle sit in consecutive lanes and share
// their first component: a segmented minimum over such runs leaves one
// atomic per run; a read of the current best skips atomics that cannot win.
__global__ void __launch_bounds__(256) k_bor_min(const uint64_t *key, const uint32_t *u,
                                                 const uint32_t *v, size_t m,
                                                 unsigned long long *best) {
  const int lane = threadIdx.x & 63;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  // the loop runs the same number of times in every lane of a wave
  const size_t base0 = (size_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u);
  for (size_t b0 = base0; b0 < m; b0 += stride) {
    const size_t c = b0 + lane;
    uint32_t cu = 0xffffffffu, cv = 0xffffffffu;
    unsigned long long k = ~0ull;
    bool live = false;
    if (c < m) {
      cu = u[c];
      cv = v[c];
      live = cu != cv;
      k = key[c];
    }
    // segmented minima over runs of equal cu and of equal cv among live
    // lanes (a home particle's candidates, or one partner's, sit together)
    const uint32_t gu = live ? cu : 0xffffffffu, gv = live ? cv : 0xffffffffu;
    unsigned long long su = live ? k : ~0ull, sv = su;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const unsigned long long ou = __shfl_down(su, d, kWave), ov = __shfl_down(sv, d, kWave);
      const uint32_t ogu = __shfl_down(gu, d, kWave), ogv = __shfl_down(gv, d, kWave);
      if (lane + d < 64 && ogu == gu && ou < su) su = ou;
      if (lane + d < 64 && ogv == gv && ov < sv) sv = ov;
    }
    const uint32_t pu = __shfl_up(gu, 1, kWave), pv = __shfl_up(gv, 1, kWave);
    const bool hu = live && (lane == 0 || pu != gu), hv = live && (lane == 0 || pv != gv);
    if (hu && best[cu] > su) atomicMin(best + cu, su);
    if (hv && best[cv] > sv) atomicMin(best + cv, sv);
  }
}

// the best edge of either end's component is a forest edge: mark it and
// hook its two components together
__global__ void k_bor_select(const uint64_t *key, const uint32_t *u, const uint32_t *v, size_t m,
                             const unsigned long long *best, uint32_t *bpar, uint8_t *sel) {
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < m;
       c += (size_t)gridDim.x * blockDim.x) {
    const uint32_t cu = u[c], cv = v[c];
    const uint64_t k = key[c];
    const bool s = cu != cv && (best[cu] == k || best[cv] == k);
    sel[c] = s ? 1 : 0;
    if (s) uf_union(bpar, cu, cv);
  }
}

// forest edges of this round -> active pairs (sorted particle indices)
__global__ void k_bor_emit(const uint64_t *key, const uint32_t *u, size_t m, const uint8_t *sel,
                           const uint32_t *pos32, const uint32_t *inv_perm, const int64_t *p_off,
                           int njobs, uint32_t *oi, uint32_t *oj, uint8_t *ot) {
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < m;
       c += (size_t)gridDim.x * blockDim.x) {
    if (!sel[c]) continue;
    const uint32_t p = pos32[c];
    const int j = job_of(p_off, njobs, (int64_t)u[c]);
    const uint64_t k = key[c];
    const uint32_t lo = (uint32_t)((k >> 31) & 0x7fffffffull), hi = (uint32_t)(k & 0x7fffffffull);
    oi[p] = inv_perm[p_off[j] + lo];
    oj[p] = inv_perm[p_off[j] + hi];
    ot[p] = (uint8_t)kPb;
  }
}

// After the round's unions (and a flatten of the parents): candidates that
// were not selected are kept only if their ends are still in different
// components, and carry the new roots.
__global__ void k_bor_relabel(const uint32_t *u, const uint32_t *v, size_t m, const uint8_t *sel,
                              const uint32_t *root, uint32_t *ru, uint32_t *rv, uint8_t *alive) {
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < m;
       c += (size_t)gridDim.x * blockDim.x) {
    uint8_t a = 0;
    uint32_t cu = 0, cv = 0;
    if (!sel[c]) {
      cu = root[u[c]];
      cv = root[v[c]];
      a = cu != cv ? 1 : 0;
    }
    alive[c] = a;
    ru[c] = cu;
    rv[c] = cv;
  }
}

__global__ void k_bor_compact(const uint64_t *key, const uint32_t *ru, const uint32_t *rv,
                              size_t m, const uint8_t *alive, const uint32_t *pos32, uint64_t *nkey,
                              uint32_t *nu, uint32_t *nv) {
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < m;
       c += (size_t)gridDim.x * blockDim.x) {
    if (!alive[c]) continue;
    const uint32_t p = pos32[c];
    nkey[p] = key[c];
    nu[p] = ru[c];
    nv[p] = rv[c];
  }
}

// Chunk-local spanning forests.  An edge that is not in the minimum
// spanning forest of some subset of the edges is the heaviest edge of a
// cycle inside that subset, so (cycle property) it is not in the forest of
// the whole graph either.  Each block takes kLocalEdges consecutive
// candidates (neighbouring homes, whose links close many triangles), finds
// their own minimum spanning forest by Boruvka rounds in LDS, and moves its
// edges to the front of its chunk; only those enter the global rounds.
// Within one job the keys of a component's edges are distinct (one key per
// particle pair), so every round's minimum edges form a forest.  Endpoints
// get local ids from an open-addressing table in LDS (at most
// 2 kLocalEdges values in kLocalSlots slots, so an insert always succeeds).
constexpr int kLocalEdges = 1024, kLocalThreads = 256, kLocalSlots = 2 * kLocalEdges;
constexpr int kLocalPer = kLocalEdges / kLocalThreads;

// root of x, halving the path (a non-root's parent only ever moves to an
// ancestor, so the store is safe beside concurrent hooks of roots)
__device__ inline uint32_t lds_find(uint32_t *par, uint32_t x) {
  for (;;) {
    const uint32_t p = __hip_atomic_load(par + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (p == x) return x;
    const uint32_t g = __hip_atomic_load(par + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (g == p) return p;
    __hip_atomic_store(par + x, g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    x = g;
  }
}
// hook the larger root under the smaller one (parents only ever decrease)
__device__ inline void lds_union(uint32_t *par, uint32_t a, uint32_t b) {
  a = lds_find(par, a);
  b = lds_find(par, b);
  while (a != b) {
    const uint32_t hi = a > b ? a : b, lo = a > b ? b : a;
    uint32_t seen = hi;
    if (__hip_atomic_compare_exchange_strong(par + hi, &seen, lo, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
      return;
    a = lds_find(par, seen);
    b = lds_find(par, lo);
  }
}
// slot of value x in the table (inserted if absent)
__device__ inline uint32_t lds_slot(uint32_t *tab, uint32_t x) {
  uint32_t h = (x * 2654435761u) >> (32 - 11);
  static_assert(kLocalSlots == 1 << 11, "hash width");
  for (;;) {
    uint32_t seen = 0xffffffffu;
    if (__hip_atomic_compare_exchange_strong(tab + h, &seen, x, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) ||
        seen == x)
      return h;
    h = (h + 1) & (kLocalSlots - 1);
  }
}

__global__ void __launch_bounds__(kLocalThreads) k_forest_local(uint64_t *key, uint32_t *u,
                                                                uint32_t *v, size_t m,
                                                                uint32_t *nkept) {
  // the endpoint table is needed only until every end has its slot; the
  // lightest edge per component takes its place afterwards
  __shared__ unsigned long long best[kLocalSlots];   // lightest edge of each component
  __shared__ uint32_t par[kLocalSlots];              // parents of the slots
  __shared__ uint32_t wsum[kLocalThreads / kWave];
  uint32_t *tab = reinterpret_cast<uint32_t *>(best);  // endpoint values
  const int tid = threadIdx.x;
  const size_t c0 = (size_t)blockIdx.x * kLocalEdges;
  const uint32_t ne = (uint32_t)(m - c0 < (size_t)kLocalEdges ? m - c0 : (size_t)kLocalEdges);
  uint32_t ea[kLocalPer], eb[kLocalPer], eu[kLocalPer], ev[kLocalPer];
  unsigned long long ek[kLocalPer];
  uint32_t live = 0, sel = 0;
  for (uint32_t x = (uint32_t)tid; x < (uint32_t)kLocalSlots; x += kLocalThreads) {
    tab[x] = 0xffffffffu;
    par[x] = x;
  }
#pragma unroll
  for (int r = 0; r < kLocalPer; ++r) {
    const uint32_t i = (uint32_t)tid + (uint32_t)r * kLocalThreads;
    ea[r] = eb[r] = 0u;
    ek[r] = ~0ull;
    if (i < ne) {
      ea[r] = u[c0 + i];
      eb[r] = v[c0 + i];
      ek[r] = key[c0 + i];
      if (ea[r] != eb[r]) live |= 1u << r;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kLocalPer; ++r) {
    eu[r] = ev[r] = 0u;
    if ((live >> r) & 1u) {
      eu[r] = lds_slot(tab, ea[r]);
      ev[r] = lds_slot(tab, eb[r]);
    }
  }
  __syncthreads();
  for (;;) {
    // roots of the live edges' ends; their components' minima start empty
    uint32_t ru[kLocalPer], rv[kLocalPer];
#pragma unroll
    for (int r = 0; r < kLocalPer; ++r) {
      ru[r] = rv[r] = 0u;
      if (!((live >> r) & 1u)) continue;
      ru[r] = lds_find(par, eu[r]);
      rv[r] = lds_find(par, ev[r]);
      if (ru[r] == rv[r]) {
        live &= ~(1u << r);
        continue;
      }
      best[ru[r]] = ~0ull;
      best[rv[r]] = ~0ull;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kLocalPer; ++r)
      if ((live >> r) & 1u) {
        atomicMin(best + ru[r], ek[r]);
        atomicMin(best + rv[r], ek[r]);
      }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kLocalPer; ++r) {
      if (!((live >> r) & 1u)) continue;
      if (best[ru[r]] == ek[r] || best[rv[r]] == ek[r]) {
        sel |= 1u << r;
        live &= ~(1u << r);
        lds_union(par, ru[r], rv[r]);
      }
    }
    if (!__syncthreads_or(live != 0)) break;
  }
  // the chunk's forest edges to the front of the chunk (every read of the
  // chunk happened above), in thread order
  const uint32_t mine = (uint32_t)__popc(sel);
  uint32_t incl = mine;
  const int lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d, kWave);
    if (lane >= d) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t base = 0, total = 0;
  for (int q = 0; q < kLocalThreads / kWave; ++q) {
    if (q < w) base += wsum[q];
    total += wsum[q];
  }
  uint32_t at = base + incl - mine;
#pragma unroll
  for (int r = 0; r < kLocalPer; ++r)
    if ((sel >> r) & 1u) {
      key[c0 + at] = ek[r];
      u[c0 + at] = ea[r];
      v[c0 + at] = eb[r];
      ++at;
    }
  if (tid == 0) nkept[blockIdx.x] = total;
}

// the kept fronts of the chunks, back to back
__global__ void k_forest_gather(const uint64_t *key, const uint32_t *u, const uint32_t *v,
                                const uint32_t *nkept, const uint32_t *off, uint64_t *nkey,
                                uint32_t *nu, uint32_t *nv) {
  const size_t c0 = (size_t)blockIdx.x * kLocalEdges;
  const uint32_t k = nkept[blockIdx.x], o = off[blockIdx.x];
  for (uint32_t i = threadIdx.x; i < k; i += blockDim.x) {
    nkey[o + i] = key[c0 + i];
    nu[o + i] = u[c0 + i];
    nv[o + i] = v[c0 + i];
  }
}

int64_t boruvka(uint64_t *key, uint32_t *u, uint32_t *v, size_t ncand, uint32_t *bpar, size_t n,
                const uint32_t *inv_perm, const int64_t *p_off, int njobs, uint32_t *out_i,
                uint32_t *out_j, uint8_t *out_t, Arena &ar, hipStream_t s) {
  if (ncand == 0) return 0;
  if (ncand > 0xffffffffull) throw Error(-6, "more than 2^32 - 1 forest candidates");
  unsigned long long *best = ar.get<unsigned long long>(n);
  uint8_t *alive = ar.get<uint8_t>(ncand);
  uint8_t *sel = ar.get<uint8_t>(ncand);
  uint32_t *pos32 = ar.get<uint32_t>(ncand);
  uint32_t *cnt = ar.get<uint32_t>(2);
  uint64_t *key2 = ar.get<uint64_t>(ncand);
  uint32_t *u2 = ar.get<uint32_t>(ncand);
  uint32_t *v2 = ar.get<uint32_t>(ncand);
  uint32_t *ru = ar.get<uint32_t>(ncand), *rv = ar.get<uint32_t>(ncand);
  uint32_t *hcnt = nullptr;
  PCC_HIP(hipHostMalloc((void **)&hcnt, 2 * sizeof(uint32_t), hipHostMallocDefault));
  int64_t emitted = 0;
  size_t m = ncand;
  try {
    {
      // the chunk-local forests' edges only
      const size_t nch = (m + kLocalEdges - 1) / kLocalEdges;
      uint32_t *nkept = ar.get<uint32_t>(nch), *off = ar.get<uint32_t>(nch);
      k_forest_local<<<(unsigned)nch, kLocalThreads, 0, s>>>(key, u, v, m, nkept);
      scan_u32_u32(nkept, off, nch, cnt, ar, s);
      k_forest_gather<<<(unsigned)nch, 128, 0, s>>>(key, u, v, nkept, off, key2, u2, v2);
      PCC_HIP(hipMemcpyAsync(hcnt, cnt, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      PCC_HIP(hipStreamSynchronize(s));
      if (getenv("PCC_VERBOSE"))
        fprintf(stderr, "[pcc] forest: %zu candidates, %u in chunk-local forests\n", m, hcnt[0]);
      m = hcnt[0];
      std::swap(key, key2);
      std::swap(u, u2);
      std::swap(v, v2);
    }
    while (m > 0) {
      const int nb = blocks_for(m, 256, 65536);
      fill_u64((uint64_t *)best, ~0ull, n, s);
      k_bor_min<<<nb, 256, 0, s>>>(key, u, v, m, best);
      k_bor_select<<<nb, 256, 0, s>>>(key, u, v, m, best, bpar, sel);
      scan_u8_u32(sel, pos32, m, cnt, ar, s);
      k_bor_emit<<<nb, 256, 0, s>>>(key, u, m, sel, pos32, inv_perm, p_off, njobs,
                                    out_i + emitted, out_j + emitted, out_t + emitted);
      launch_flatten(bpar, n, s);
      k_bor_relabel<<<nb, 256, 0, s>>>(u, v, m, sel, bpar, ru, rv, alive);
      scan_u8_u32(alive, pos32, m, cnt + 1, ar, s);
      k_bor_compact<<<nb, 256, 0, s>>>(key, ru, rv, m, alive, pos32, key2, u2, v2);
      PCC_HIP(hipMemcpyAsync(hcnt, cnt, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      PCC_HIP(hipStreamSynchronize(s));
      emitted += hcnt[0];
      if (getenv("PCC_VERBOSE"))
        fprintf(stderr, "[pcc] forest round: %zu candidates, %u selected, %u left\n", m, hcnt[0],
                hcnt[1]);
      if (hcnt[0] == 0 && hcnt[1] != 0)
        throw Error(-3, "spanning forest made no progress");
      m = hcnt[1];
      std::swap(key, key2);
      std::swap(u, u2);
      std::swap(v, v2);
    }
  } catch (...) {
    hipHostFree(hcnt);
    throw;
  }
  hipHostFree(hcnt);
  return emitted;
}

}  // namespace pcc
