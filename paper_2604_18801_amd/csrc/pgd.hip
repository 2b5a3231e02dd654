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

__global__ void k_incid(const uint32_t *a_i, const uint32_t *a_j, const uint8_t *a_t, size_t na,
                        const uint32_t *eid, uint32_t *keys, uint32_t *vals) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < na;
       p += (size_t)gridDim.x * blockDim.x) {
    const uint32_t ri = eid[a_i[p]], rj = eid[a_j[p]];
    const uint32_t t = a_t[p] == 3 ? 0x80000000u : 0u;
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
__global__ void k_take_pairs(const uint32_t *a_i, const uint32_t *a_j, const uint8_t *a_t,
                             const uint32_t *idx, size_t na, uint32_t *b_i, uint32_t *b_j,
                             uint8_t *b_t) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < na;
       p += (size_t)gridDim.x * blockDim.x) {
    const uint32_t q = idx[p];
    b_i[p] = a_i[q];
    b_j[p] = a_j[q];
    b_t[p] = a_t[q];
  }
}

// Orders the active pairs by (smaller job-local index, larger one) with two
// stable radix sorts.  The stable sort of their incidences by row that
// follows then leaves every row in increasing partner index: the order in
// which the gradient of each particle is summed.
void sort_pairs(uint32_t *a_i, uint32_t *a_j, uint8_t *a_t, size_t na, const float4 *pos,
                int id_bits, Arena &ar, hipStream_t s) {
  if (na < 2) return;
  uint32_t *lo = ar.get<uint32_t>(na), *hi = ar.get<uint32_t>(na), *idx = ar.get<uint32_t>(na);
  const int nb = blocks_for(na, 256, 65536);
  k_pair_keys<<<nb, 256, 0, s>>>(a_i, a_j, na, pos, lo, hi, idx);
  radix_sort_u32(hi, idx, na, id_bits, ar, s);
  k_take_u32<<<nb, 256, 0, s>>>(lo, idx, na, hi);
  radix_sort_u32(hi, idx, na, id_bits, ar, s);
  uint32_t *b_i = ar.get<uint32_t>(na), *b_j = ar.get<uint32_t>(na);
  uint8_t *b_t = ar.get<uint8_t>(na);
  k_take_pairs<<<nb, 256, 0, s>>>(a_i, a_j, a_t, idx, na, b_i, b_j, b_t);
  PCC_HIP(hipMemcpyAsync(a_i, b_i, na * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
  PCC_HIP(hipMemcpyAsync(a_j, b_j, na * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
  PCC_HIP(hipMemcpyAsync(a_t, b_t, na, hipMemcpyDeviceToDevice, s));
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

void build_csr(const uint32_t *a_i, const uint32_t *a_j, const uint8_t *a_t, size_t na,
               const uint32_t *eid, uint32_t ne, uint32_t *row_ptr, uint32_t *col, Arena &ar,
               hipStream_t s) {
  if (!na) {
    PCC_HIP(hipMemsetAsync(row_ptr, 0, sizeof(uint32_t) * ((size_t)ne + 1), s));
    return;
  }
  const size_t m = 2 * na;
  if (m > 0xffffffffull) throw Error(-6, "more than 2^31 active pairs in one call");
  uint32_t *keys = ar.get<uint32_t>(m);
  k_incid<<<blocks_for(na, 256, 65536), 256, 0, s>>>(a_i, a_j, a_t, na, eid, keys, col);
  radix_sort_u32(keys, col, m, bits_for(ne ? ne - 1 : 0), ar, s);
  k_row_ptr<<<blocks_for(m, 256, 65536), 256, 0, s>>>(keys, m, ne, row_ptr);
}

__global__ void k_pgd_init(const uint32_t *e_list, size_t ne, const float4 *pos, const float4 *rec,
                           double4 *P0, float4 *xo, double *m, double *v) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne;
       e += (size_t)gridDim.x * blockDim.x) {
    const uint32_t k = e_list[e];
    const float4 r = rec[k];
    P0[e] = make_double4((double)r.x, (double)r.y, (double)r.z, 0.0);
    xo[e] = pos[k];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      m[a * ne + e] = 0.0;
      v[a * ne + e] = 0.0;
    }
  }
}

void launch_pgd_init(const uint32_t *e_list, size_t ne, const float4 *pos, const float4 *rec,
                     double4 *P0, float4 *xo, double *m, double *v, hipStream_t s) {
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
__device__ inline double wrapd(double d, double L, double hL) {
  if (d > hL)
    d -= L;
  else if (d < -hL)
    d += L;
  return d;
}

__device__ inline unsigned long long wsum(unsigned long long v) {
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

struct RowConst {
  double L0, L1, L2, h0, h1, h2, bm, bp, bm2, bp2, scale;
};

__device__ inline RowConst row_const(const JobDev &J) {
  RowConst c;
  c.L0 = J.L[0];
  c.L1 = J.L[1];
  c.L2 = J.L[2];
  c.h0 = J.hL[0];
  c.h1 = J.hL[1];
  c.h2 = J.hL[2];
  c.bm = J.bm;
  c.bp = J.bp;
  c.bm2 = J.bm2;
  c.bp2 = J.bp2;
  c.scale = J.loss_scale;
  return c;
}

constexpr int kPgdWaves = 4;
constexpr int kPgdBlocks = 2048;  // resident waves: 8192, about 8 per SIMD

// flush of the per-job violation count and fixed-point loss of one wave
__device__ inline void flush_counts(JobLoop *loop, int job, unsigned long long &viol,
                                    unsigned long long &lossq) {
  const unsigned long long sv = wsum(viol), sl = wsum(lossq);
  if ((threadIdx.x & 63) == 0 && job >= 0) {
    if (sv) atomicAdd(&loop[job].viol_acc, sv);
    if (sl) atomicAdd(&loop[job].loss_acc, sl);
  }
  viol = 0;
  lossq = 0;
}

// Each wave walks tiles of up to 64 consecutive rows of one job (tiles never
// straddle two jobs, so the job and its constants are wave-uniform).  The
// incidences of a tile (a contiguous range of the column array) are spread
// over the 64 lanes, 64 at a time: each lane gathers one partner, evaluates
// one constraint and leaves its gradient term in LDS; then each row's owner
// lane adds the terms of its row in column order (increasing partner
// index).  Finally every lane takes the Adam step and the projection of its
// own row.  Violation counts stay in registers until the wave moves to
// another job or finishes.
#ifndef PCC_PGD_MIN_WAVES
#define PCC_PGD_MIN_WAVES 1
#endif
__global__ void __launch_bounds__(64 * kPgdWaves, PCC_PGD_MIN_WAVES) k_pgd_step(PgdBufs B) {
  __shared__ double4 s_self[kPgdWaves][64];
  __shared__ double s_term[kPgdWaves][3][64];
  __shared__ uint32_t s_rp[kPgdWaves][65];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t nwaves = (int64_t)gridDim.x * kPgdWaves;
  unsigned long long viol = 0, lossq = 0;
  int cjob = -1;  // job whose counts are held in viol / lossq
  for (int64_t tile = (int64_t)blockIdx.x * kPgdWaves + w; tile < B.ntiles; tile += nwaves) {
    const int job = __builtin_amdgcn_readfirstlane(job_of(B.tile_off, B.njobs, tile));
    if (B.loop[job].done) continue;
    if (job != cjob) {
      flush_counts(B.loop, cjob, viol, lossq);
      cjob = job;
    }
    const JobDev &J = B.jobs[job];
    const int64_t e0 = B.e_off[job] + (tile - B.tile_off[job]) * 64;
    const int64_t left = B.e_off[job + 1] - e0;
    const int nrow = (int)(left < 64 ? left : 64);
    const bool valid = lane < nrow;
    const size_t e = (size_t)e0 + lane;
    const int cur = (int)(B.loop[job].t & 1);
    const double4 *__restrict__ Pc = cur ? B.P1 : B.P0;
    double4 *__restrict__ Pn = cur ? B.P0 : B.P1;
    const double L0 = J.L[0], L1 = J.L[1], L2 = J.L[2];
    const double h0 = J.hL[0], h1 = J.hL[1], h2 = J.hL[2];
    const double bm = J.bm, bp = J.bp, bm2 = J.bm2, bp2 = J.bp2, scale = J.loss_scale;
    // the row's own state, loaded ahead of the gathers
    double4 pe = make_double4(0.0, 0.0, 0.0, 0.0);
    float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
    double mo[3] = {0.0, 0.0, 0.0}, vo[3] = {0.0, 0.0, 0.0};
    if (valid) {
      pe = Pc[e];
      x = B.xo[e];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        mo[k] = B.m[(size_t)k * B.ne + e];
        vo[k] = B.v[(size_t)k * B.ne + e];
      }
    }
    s_self[w][lane] = pe;
    s_rp[w][lane] = valid ? B.row_ptr[e] : 0xffffffffu;
    if (lane == 0) s_rp[w][64] = B.row_ptr[e0 + nrow];
    wave_sync();
    const uint32_t qs = s_rp[w][0], qe = s_rp[w][64];
    const uint32_t my_q0 = valid ? s_rp[w][lane] : qe;
    const uint32_t my_q1 = valid ? (lane + 1 < nrow ? s_rp[w][lane + 1] : qe) : qe;
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (uint32_t c0 = qs; c0 < qe; c0 += 64) {
      const uint32_t q = c0 + lane;
      double tx = 0.0, ty = 0.0, tz = 0.0;
      if (q < qe) {
        // owner row of incidence q: last r with s_rp[r] <= q
        int lo = 0, hi = nrow - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_rp[w][mid] <= q)
            lo = mid;
          else
            hi = mid - 1;
        }
        const int r = lo;
        const uint32_t col = B.col[q];
        const uint32_t o = col & 0x7fffffffu;
        const double4 me = s_self[w][r];
        const double4 po = Pc[o];
        const double dx = wrapd(me.x - po.x, L0, h0);
        const double dy = wrapd(me.y - po.y, L1, h1);
        const double dz = wrapd(me.z - po.z, L2, h2);
        const double d2 = (dx * dx + dy * dy) + dz * dz;
        const size_t er = (size_t)e0 + r;
        bool hit = false;
        double h = 0.0;
        if (!(col >> 31)) {
          // potentially broken: an original link pulled back inside b - delta_t
          if (d2 > bm2) {
            const double d = sqrt(d2);
            h = d - bm;
            tx = 2.0 * h * (dx / d);
            ty = 2.0 * h * (dy / d);
            tz = 2.0 * h * (dz / d);
            hit = true;
          }
        } else if (d2 <= bp2) {
          // potentially created: an original non-link pushed beyond b + delta_t
          const double d = sqrt(d2);
          h = bp - d;
          double ux, uy, uz;
          if (d > 0.0) {
            ux = dx / d;
            uy = dy / d;
            uz = dz / d;
          } else {
            // coincident points: take the direction of the original pair
            const float4 a = B.xo[er], b = B.xo[o];
            const double ox = wrapd((double)a.x - (double)b.x, L0, h0);
            const double oy = wrapd((double)a.y - (double)b.y, L1, h1);
            const double oz = wrapd((double)a.z - (double)b.z, L2, h2);
            const double od = sqrt((ox * ox + oy * oy) + oz * oz);
            ux = ox / od;
            uy = oy / od;
            uz = oz / od;
          }
          tx = -(2.0 * h * ux);
          ty = -(2.0 * h * uy);
          tz = -(2.0 * h * uz);
          hit = true;
        }
        if (hit && o > er) {
          viol++;
          lossq += (unsigned long long)(h * h * scale);
        }
      }
      s_term[w][0][lane] = tx;
      s_term[w][1][lane] = ty;
      s_term[w][2][lane] = tz;
      wave_sync();
      // the owner adds the terms of its row that fall in this chunk, in order
      const uint32_t a = my_q0 > c0 ? my_q0 : c0;
      const uint32_t b = my_q1 < c0 + 64 ? my_q1 : c0 + 64;
      for (uint32_t t = a; t < b; ++t) {
        gx += s_term[w][0][t - c0];
        gy += s_term[w][1][t - c0];
        gz += s_term[w][2][t - c0];
      }
      wave_sync();
    }
    if (valid) {
      const double bc1 = B.loop[job].bc1, bc2 = B.loop[job].bc2;
      const double g[3] = {gx, gy, gz};
      const double p[3] = {pe.x, pe.y, pe.z};
      const double xs[3] = {(double)x.x, (double)x.y, (double)x.z};
      double np[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double r;
        if (J.optimizer == 1) {
          r = p[k] - J.lr * g[k];
        } else {
          const size_t ia = (size_t)k * B.ne + e;
          const double m = J.beta1 * mo[k] + J.one_m_beta1 * g[k];
          const double v = J.beta2 * vo[k] + J.one_m_beta2 * g[k] * g[k];
          B.m[ia] = m;
          B.v[ia] = v;
          const double mh = m / bc1;
          const double vh = v / bc2;
          r = p[k] - J.lr * mh / (sqrt(vh) + J.adam_eps);
        }
        np[k] = fmin(fmax(r, xs[k] - J.xi_p), xs[k] + J.xi_p);
      }
      Pn[e] = make_double4(np[0], np[1], np[2], 0.0);
    }
    wave_sync();  // LDS of this tile is reused by the next one
  }
  flush_counts(B.loop, cjob, viol, lossq);
}

__global__ void k_pgd_finalize(PgdBufs B) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= B.njobs) return;
  JobLoop &L = B.loop[j];
  if (L.done) return;
  const JobDev &J = B.jobs[j];
  const unsigned long long viol = L.viol_acc, lq = L.loss_acc;
  L.viol_acc = 0;
  L.loss_acc = 0;
  if (!L.have0) {
    L.viol0 = viol;
    L.loss0 = lq;
    L.have0 = 1;
  }
  L.viol_last = viol;
  L.loss_last = lq;
  const bool conv = J.loss_tol > 0.0 ? ((double)lq / J.loss_scale <= J.loss_tol) : (viol == 0);
  if (conv || L.t >= J.max_iters) {
    L.done = 1;
    L.status = conv ? 0 : 1;
    atomicSub(B.n_active, 1);
    return;
  }
  L.t += 1;
  L.bc1 = J.bc_tab[L.t + 1].x;
  L.bc2 = J.bc_tab[L.t + 1].y;
}

void launch_pgd_step(const PgdBufs &b, hipStream_t s) {
  if (b.ne)
    k_pgd_step<<<blocks_for(b.ne, 64 * kPgdWaves, kPgdBlocks), 64 * kPgdWaves, 0, s>>>(b);
}
void launch_pgd_finalize(const PgdBufs &b, hipStream_t s) {
  k_pgd_finalize<<<(b.njobs + 255) / 256, 256, 0, s>>>(b);
}

}  // namespace pcc
