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

// find with path halving: every parent pointer only ever moves to an ancestor
__device__ inline uint32_t uf_find(uint32_t *par, uint32_t x) {
  for (;;) {
    const uint32_t p = ld_par(par, x);
    if (p == x) return x;
    const uint32_t gp = ld_par(par, p);
    if (gp == p) return p;
    st_par(par, x, gp);
    x = gp;
  }
}

// hook the larger root under the smaller one with a compare-and-swap; retry
// from the new roots when another thread got there first
__device__ inline void uf_union(uint32_t *par, uint32_t a, uint32_t b) {
  for (;;) {
    a = uf_find(par, a);
    b = uf_find(par, b);
    if (a == b) return;
    if (a < b) {
      const uint32_t t = a;
      a = b;
      b = t;
    }
    uint32_t expected = a;
    if (__hip_atomic_compare_exchange_strong(par + a, &expected, b, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return;
  }
}

// ----------------------------------------------------------------------------
// wave-aggregated per-job counters
// ----------------------------------------------------------------------------
__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

template <int K>
__device__ inline void job_add(unsigned long long *ctr, int job, bool valid,
                               const unsigned long long (&v)[K]) {
  const int jv = valid ? job : -1;
  uint64_t todo = __ballot(valid);
  const int lane = threadIdx.x & 63;
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int lj = __shfl(jv, leader, kWave);
    const uint64_t grp = __ballot(jv == lj);
#pragma unroll
    for (int c = 0; c < K; ++c) {
      const unsigned long long s = wave_sum_u64(jv == lj ? v[c] : 0ull);
      if (lane == leader && s) atomicAdd(ctr + (size_t)lj * K + c, s);
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
  float rv2f;
  int mode;
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
  q.rv2f = J.rv2_f32;
  q.mode = J.mode;
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

template <int PASS>
__global__ void __launch_bounds__(256) k_pairs(PairBufs B) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = k < B.n;
  const int job = valid ? job_of(B.p_off, B.njobs, (int64_t)k) : 0;
  unsigned long long cnt[3] = {0ull, 0ull, 0ull};  // safe, pb, pc
  if (valid) {
    const JobPair q = load_job(B.jobs[job]);
    const float4 pi = B.pos[k];
    const uint32_t cell = B.cell_of[k];
    uint32_t sk = 0, fk = 0;
    float4 ri = make_float4(0.f, 0.f, 0.f, 0.f);
    if (PASS >= 2) {
      sk = B.safe_par[k];
      fk = B.fof_par[k];
    }
    if (PASS == 3) ri = B.rec[k];
    uint64_t wa = PASS == 3 ? B.off_a[k] : 0, wf = PASS == 3 ? B.off_f[k] : 0;
    uint32_t ca = 0, cf = 0;
    for (int s = 0; s < 14; ++s) {
      uint32_t j0, j1;
      if (s == 0) {
        j0 = (uint32_t)k + 1;
        j1 = B.cell_start[cell + 1];
      } else {
        const int32_t nb = B.nbr[(size_t)cell * 13 + s - 1];
        if (nb < 0) continue;
        j0 = B.cell_start[nb];
        j1 = B.cell_start[nb + 1];
      }
      for (uint32_t j = j0; j < j1; ++j) {
        const float4 pj = B.pos[j];
        const float dx = wrap_f(pi.x - pj.x, q.Lf[0], q.hLf[0]);
        const float dy = wrap_f(pi.y - pj.y, q.Lf[1], q.hLf[1]);
        const float dz = wrap_f(pi.z - pj.z, q.Lf[2], q.hLf[2]);
        const float d2f = (dx * dx + dy * dy) + dz * dz;
        if (d2f > q.rv2f) continue;
        const double d2 = dist2_exact(pi, pj, q);
        if (d2 > q.rv2) continue;
        const int cls = d2 <= q.rs2 ? kSafe : (d2 <= q.b2 ? kPb : kPc);
        if (PASS == 1) {
          if (cls == kSafe) {
            cnt[0]++;
            uf_union(B.safe_par, (uint32_t)k, j);
            uf_union(B.fof_par, (uint32_t)k, j);
          } else if (cls == kPb) {
            cnt[1]++;
            ca++;
            uf_union(B.fof_par, (uint32_t)k, j);
          } else {
            cnt[2]++;
            ca++;
          }
          continue;
        }
        if (cls == kSafe) continue;
        bool to_a = false, to_f = false;
        if (q.mode == 0) {
          to_a = true;
        } else if (q.mode == 1) {
          to_a = B.safe_par[j] != sk;
        } else if (cls == kPc) {
          to_a = B.fof_par[j] != fk;
        } else {
          to_f = B.safe_par[j] != sk;
        }
        if (PASS == 2) {
          ca += to_a;
          cf += to_f;
        } else {
          if (to_a) {
            B.a_i[wa] = (uint32_t)k;
            B.a_j[wa] = j;
            B.a_t[wa] = (uint8_t)cls;
            wa++;
          }
          if (to_f) {
            const float4 rj = B.rec[j];
            const double ex = wrap_d((double)ri.x - (double)rj.x, q.L[0], q.hL[0]);
            const double ey = wrap_d((double)ri.y - (double)rj.y, q.L[1], q.hL[1]);
            const double ez = wrap_d((double)ri.z - (double)rj.z, q.L[2], q.hL[2]);
            const uint64_t viol0 = ((ex * ex + ey * ey) + ez * ez) > q.bm2 ? 1ull : 0ull;
            const uint32_t li = __float_as_uint(pi.w), lj = __float_as_uint(pj.w);
            const uint64_t lo = li < lj ? li : lj, hi = li < lj ? lj : li;
            B.f_key[wf] = (viol0 << 62) | (lo << 31) | hi;
            B.f_u[wf] = sk;
            B.f_v[wf] = B.safe_par[j];
            wf++;
          }
        }
      }
    }
    if (PASS == 1) B.cnt_a[k] = ca;
    if (PASS == 2) {
      B.cnt_a[k] = ca;
      B.cnt_f[k] = cf;
    }
  }
  if (PASS == 1) job_add<3>(B.job_counts, job, valid, cnt);
}

void launch_pair_pass1(const PairBufs &b, hipStream_t s) {
  if (b.n) k_pairs<1><<<blocks_for(b.n, 256, 1 << 30), 256, 0, s>>>(b);
}
void launch_pair_count(const PairBufs &b, hipStream_t s) {
  if (b.n) k_pairs<2><<<blocks_for(b.n, 256, 1 << 30), 256, 0, s>>>(b);
}
void launch_pair_write(const PairBufs &b, hipStream_t s) {
  if (b.n) k_pairs<3><<<blocks_for(b.n, 256, 1 << 30), 256, 0, s>>>(b);
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
__global__ void k_minid(const uint32_t *root, const float4 *pos, size_t n, uint32_t *minid) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x)
    atomicMin(minid + root[k], __float_as_uint(pos[k].w));
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
__global__ void k_bor_min(const uint64_t *key, const uint32_t *u, const uint32_t *v, size_t m,
                          uint32_t *bpar, unsigned long long *best, uint8_t *alive) {
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < m;
       c += (size_t)gridDim.x * blockDim.x) {
    const uint32_t cu = uf_find(bpar, u[c]), cv = uf_find(bpar, v[c]);
    if (cu == cv) {
      alive[c] = 0;
      continue;
    }
    alive[c] = 1;
    atomicMin(best + cu, (unsigned long long)key[c]);
    atomicMin(best + cv, (unsigned long long)key[c]);
  }
}

__global__ void k_bor_mark(const uint64_t *key, const uint32_t *u, const uint32_t *v, size_t m,
                           uint32_t *bpar, const unsigned long long *best, uint8_t *alive,
                           uint8_t *sel) {
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < m;
       c += (size_t)gridDim.x * blockDim.x) {
    uint8_t s = 0;
    if (alive[c]) {
      const uint32_t cu = uf_find(bpar, u[c]), cv = uf_find(bpar, v[c]);
      s = (best[cu] == key[c] || best[cv] == key[c]) ? 1 : 0;
      if (s) alive[c] = 0;
    }
    sel[c] = s;
  }
}

__global__ void k_bor_union(const uint32_t *u, const uint32_t *v, size_t m, const uint8_t *sel,
                            uint32_t *bpar) {
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < m;
       c += (size_t)gridDim.x * blockDim.x)
    if (sel[c]) uf_union(bpar, u[c], v[c]);
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

__global__ void k_bor_compact(const uint64_t *key, const uint32_t *u, const uint32_t *v, size_t m,
                              const uint8_t *alive, const uint32_t *pos32, uint64_t *nkey,
                              uint32_t *nu, uint32_t *nv) {
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < m;
       c += (size_t)gridDim.x * blockDim.x) {
    if (!alive[c]) continue;
    const uint32_t p = pos32[c];
    nkey[p] = key[c];
    nu[p] = u[c];
    nv[p] = v[c];
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
  uint32_t *hcnt = nullptr;
  PCC_HIP(hipHostMalloc((void **)&hcnt, 2 * sizeof(uint32_t), hipHostMallocDefault));
  int64_t emitted = 0;
  size_t m = ncand;
  try {
    while (m > 0) {
      const int nb = blocks_for(m, 256, 65536);
      fill_u64((uint64_t *)best, ~0ull, n, s);
      k_bor_min<<<nb, 256, 0, s>>>(key, u, v, m, bpar, best, alive);
      k_bor_mark<<<nb, 256, 0, s>>>(key, u, v, m, bpar, best, alive, sel);
      k_bor_union<<<nb, 256, 0, s>>>(u, v, m, sel, bpar);
      scan_u8_u32(sel, pos32, m, cnt, ar, s);
      k_bor_emit<<<nb, 256, 0, s>>>(key, u, m, sel, pos32, inv_perm, p_off, njobs,
                                    out_i + emitted, out_j + emitted, out_t + emitted);
      scan_u8_u32(alive, pos32, m, cnt + 1, ar, s);
      k_bor_compact<<<nb, 256, 0, s>>>(key, u, v, m, alive, pos32, key2, u2, v2);
      PCC_HIP(hipMemcpyAsync(hcnt, cnt, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      PCC_HIP(hipStreamSynchronize(s));
      emitted += hcnt[0];
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
