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

void build_csr(const uint32_t *a_i, const uint32_t *a_j, const uint8_t *a_t, size_t na,
               const uint8_t *is_e, const uint32_t *eid, size_t n, uint32_t ne, uint32_t *e_list,
               uint32_t *row_ptr, uint32_t *col, Arena &ar, hipStream_t s) {
  if (n) k_e_list<<<blocks_for(n, 256, 65536), 256, 0, s>>>(is_e, eid, n, e_list);
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

__global__ void __launch_bounds__(256) k_pgd_step(PgdBufs B) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = e < B.ne;
  const int job = valid ? job_of(B.e_off, B.njobs, (int64_t)e) : 0;
  const bool active = valid && !B.loop[job].done;
  unsigned long long viol = 0, lossq = 0;
  if (active) {
    const JobDev &J = B.jobs[job];
    const JobLoop &LP = B.loop[job];
    const int cur = (int)(LP.t & 1);
    const double4 *__restrict__ Pc = cur ? B.P1 : B.P0;
    double4 *__restrict__ Pn = cur ? B.P0 : B.P1;
    const double L0 = J.L[0], L1 = J.L[1], L2 = J.L[2];
    const double h0 = J.hL[0], h1 = J.hL[1], h2 = J.hL[2];
    const double bm = J.bm, bp = J.bp, bm2 = J.bm2, bp2 = J.bp2, scale = J.loss_scale;
    const double4 pe = Pc[e];
    double gx = 0.0, gy = 0.0, gz = 0.0;
    const uint32_t q0 = B.row_ptr[e], q1 = B.row_ptr[e + 1];
    for (uint32_t q = q0; q < q1; ++q) {
      const uint32_t c = B.col[q];
      const uint32_t o = c & 0x7fffffffu;
      const double4 po = Pc[o];
      const double dx = wrapd(pe.x - po.x, L0, h0);
      const double dy = wrapd(pe.y - po.y, L1, h1);
      const double dz = wrapd(pe.z - po.z, L2, h2);
      const double d2 = (dx * dx + dy * dy) + dz * dz;
      if (!(c >> 31)) {
        // potentially broken: an original link pulled back inside b - delta_t
        if (d2 > bm2) {
          const double d = sqrt(d2);
          const double h = d - bm;
          gx += 2.0 * h * (dx / d);
          gy += 2.0 * h * (dy / d);
          gz += 2.0 * h * (dz / d);
          if (o > e) {
            viol++;
            lossq += (unsigned long long)(h * h * scale);
          }
        }
      } else {
        // potentially created: an original non-link pushed beyond b + delta_t
        if (d2 <= bp2) {
          const double d = sqrt(d2);
          const double h = bp - d;
          double ux, uy, uz;
          if (d > 0.0) {
            ux = dx / d;
            uy = dy / d;
            uz = dz / d;
          } else {
            // coincident points: take the direction of the original pair
            const float4 a = B.xo[e], b = B.xo[o];
            const double ox = wrapd((double)a.x - (double)b.x, L0, h0);
            const double oy = wrapd((double)a.y - (double)b.y, L1, h1);
            const double oz = wrapd((double)a.z - (double)b.z, L2, h2);
            const double od = sqrt((ox * ox + oy * oy) + oz * oz);
            ux = ox / od;
            uy = oy / od;
            uz = oz / od;
          }
          gx -= 2.0 * h * ux;
          gy -= 2.0 * h * uy;
          gz -= 2.0 * h * uz;
          if (o > e) {
            viol++;
            lossq += (unsigned long long)(h * h * scale);
          }
        }
      }
    }
    // optimiser step and projection onto the box around the original
    const float4 x = B.xo[e];
    const double g[3] = {gx, gy, gz};
    const double p[3] = {pe.x, pe.y, pe.z};
    const double xs[3] = {(double)x.x, (double)x.y, (double)x.z};
    double np[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double r;
      if (J.optimizer == 1) {
        r = p[a] - J.lr * g[a];
      } else {
        const size_t ia = (size_t)a * B.ne + e;
        const double m = J.beta1 * B.m[ia] + J.one_m_beta1 * g[a];
        const double v = J.beta2 * B.v[ia] + J.one_m_beta2 * g[a] * g[a];
        B.m[ia] = m;
        B.v[ia] = v;
        const double mh = m / LP.bc1;
        const double vh = v / LP.bc2;
        r = p[a] - J.lr * mh / (sqrt(vh) + J.adam_eps);
      }
      np[a] = fmin(fmax(r, xs[a] - J.xi_p), xs[a] + J.xi_p);
    }
    Pn[e] = make_double4(np[0], np[1], np[2], 0.0);
  }
  // per-job accumulation of the violation count and fixed-point loss
  const int jv = active ? job : -1;
  uint64_t todo = __ballot(active);
  const int lane = threadIdx.x & 63;
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int lj = __shfl(jv, leader, kWave);
    const uint64_t grp = __ballot(jv == lj);
    const unsigned long long sv = wsum(jv == lj ? viol : 0ull);
    const unsigned long long sl = wsum(jv == lj ? lossq : 0ull);
    if (lane == leader) {
      if (sv) atomicAdd(&B.loop[lj].viol_acc, sv);
      if (sl) atomicAdd(&B.loop[lj].loss_acc, sl);
    }
    todo &= ~grp;
  }
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
  if (b.ne) k_pgd_step<<<blocks_for(b.ne, 256, 1 << 30), 256, 0, s>>>(b);
}
void launch_pgd_finalize(const PgdBufs &b, hipStream_t s) {
  k_pgd_finalize<<<(b.njobs + 255) / 256, 256, 0, s>>>(b);
}

}  // namespace pcc
