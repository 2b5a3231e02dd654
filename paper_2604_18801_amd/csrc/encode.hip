// Edit encoding (Alg. 1 last lines; Sec. 3.3 "Compaction, quantization, and
// lossless compression"): edits = final - reconstruction in float64, a flag
// per particle with a non-zero edit, m-bit uniform codes of the three edit
// components of every flagged particle (planar x | y | z, increasing particle
// index), their histogram, and the Huffman bit-packing of the codes with a
// host-built canonical code table.
#include "kernels.hpp"

namespace pcc {

// final position of row e of job `job`
__device__ inline double3 final_pos(const EncBufs &b, int job, size_t e) {
  double3 p;
  load_p((b.loop[job].t & 1) ? b.P1 : b.P0, e, p.x, p.y, p.z);
  return p;
}

__global__ void k_edit_flags(EncBufs B) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < B.ne;
       e += (size_t)gridDim.x * blockDim.x) {
    const int j = job_of(B.e_off, B.njobs, (int64_t)e);
    const uint32_t k = B.e_list[e];
    const double3 p = final_pos(B, j, e);
    const float4 r = B.rec[k];
    const bool moved = (p.x - (double)r.x) != 0.0 || (p.y - (double)r.y) != 0.0 ||
                       (p.z - (double)r.z) != 0.0;
    B.flag8[B.p_off[j] + __float_as_uint(B.pos[k].w)] = moved ? 1 : 0;
  }
}

void launch_edit_flags(const EncBufs &b, hipStream_t s) {
  fill_u8(b.flag8, 0, b.n, s);
  if (b.ne) k_edit_flags<<<blocks_for(b.ne, 256, 65536), 256, 0, s>>>(b);
}

// code = clamp(rint((edit + 2 xi) / step), 0, 2^m - 1); m = 32 codes are
// split into a low and a high 16-bit symbol
__global__ void k_edit_codes(EncBufs B, const uint32_t *fstart) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < B.ne;
       e += (size_t)gridDim.x * blockDim.x) {
    const int j = job_of(B.e_off, B.njobs, (int64_t)e);
    const uint32_t k = B.e_list[e];
    const int64_t g = B.p_off[j] + __float_as_uint(B.pos[k].w);
    if (!B.flag8[g]) continue;
    const JobDev &J = B.jobs[j];
    const double3 p = final_pos(B, j, e);
    const float4 r = B.rec[k];
    const double d[3] = {p.x - (double)r.x, p.y - (double)r.y, p.z - (double)r.z};
    const int per = J.m_bits == 32 ? 2 : 1;
    const uint64_t nf = (B.sym_off[j + 1] - B.sym_off[j]) / (uint64_t)(3 * per);
    const uint64_t at = (uint64_t)(B.fpos[g] - fstart[j]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double qv = rint((d[a] + J.qoffset) / J.qstep);
      qv = fmin(fmax(qv, 0.0), J.qmax);
      const uint64_t code = (uint64_t)qv;
      const uint64_t base = B.sym_off[j] + (uint64_t)a * per * nf + per * at;
      if (per == 2) {
        B.sym[base] = (uint16_t)(code & 0xffffu);
        B.sym[base + 1] = (uint16_t)(code >> 16);
      } else {
        B.sym[base] = (uint16_t)code;
      }
    }
  }
}

void launch_edit_codes(const EncBufs &b, const uint32_t *fstart, hipStream_t s) {
  if (b.ne) k_edit_codes<<<blocks_for(b.ne, 256, 65536), 256, 0, s>>>(b, fstart);
}

__global__ void k_flag_bytes(const uint8_t *flag8, const int64_t *p_off, const uint64_t *fb_off,
                             int njobs, size_t nbytes, uint8_t *bytes) {
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < nbytes;
       q += (size_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (fb_off[mid] <= q)
        lo = mid;
      else
        hi = mid - 1;
    }
    const int64_t n = p_off[lo + 1] - p_off[lo];
    const int64_t first = (int64_t)(q - fb_off[lo]) * 8;
    uint32_t v = 0;
    for (int t = 0; t < 8; ++t)
      if (first + t < n && flag8[p_off[lo] + first + t]) v |= 1u << t;
    bytes[q] = (uint8_t)v;
  }
}

void launch_flag_bytes(const uint8_t *flag8, const int64_t *p_off, const uint64_t *fb_off,
                       int njobs, size_t nbytes, uint8_t *bytes, hipStream_t s) {
  if (nbytes)
    k_flag_bytes<<<blocks_for(nbytes, 256, 65536), 256, 0, s>>>(flag8, p_off, fb_off, njobs,
                                                                nbytes, bytes);
}

__device__ inline int job_of_u64(const uint64_t *off, int njobs, uint64_t g) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// table entry: bit-reversed canonical code in the low 24 bits, length above
__global__ void k_sym_len(const uint16_t *sym, size_t nsym, const uint64_t *sym_off, int njobs,
                          const uint32_t *table, uint32_t *len) {
  for (size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x; s < nsym;
       s += (size_t)gridDim.x * blockDim.x) {
    const int j = job_of_u64(sym_off, njobs, s);
    len[s] = table[(size_t)j * 65536 + sym[s]] >> 24;
  }
}

void launch_sym_lengths(const uint16_t *sym, size_t nsym, const uint64_t *sym_off, int njobs,
                        const uint32_t *table, uint32_t *len, hipStream_t s) {
  if (nsym)
    k_sym_len<<<blocks_for(nsym, 256, 65536), 256, 0, s>>>(sym, nsym, sym_off, njobs, table, len);
}

// each symbol ORs its code bits into the job's word-aligned bitstream; bit q
// of a job's stream is bit (q mod 32) of its little-endian word q / 32
__global__ void k_pack(const uint16_t *sym, size_t nsym, const uint64_t *sym_off, int njobs,
                       const uint32_t *table, const uint64_t *bitpos, const uint64_t *job_bit0,
                       const uint64_t *job_word0, uint32_t *words) {
  for (size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x; s < nsym;
       s += (size_t)gridDim.x * blockDim.x) {
    const int j = job_of_u64(sym_off, njobs, s);
    const uint32_t t = table[(size_t)j * 65536 + sym[s]];
    const uint64_t pos = bitpos[s] - job_bit0[j];
    const uint64_t w = job_word0[j] + (pos >> 5);
    const uint64_t v = (uint64_t)(t & 0xffffffu) << (pos & 31);
    if ((uint32_t)v) atomicOr(words + w, (uint32_t)v);
    if ((uint32_t)(v >> 32)) atomicOr(words + w + 1, (uint32_t)(v >> 32));
  }
}

void launch_pack_bits(const uint16_t *sym, size_t nsym, const uint64_t *sym_off, int njobs,
                      const uint32_t *table, const uint64_t *bitpos, const uint64_t *job_bit0,
                      const uint64_t *job_word0, uint32_t *words, hipStream_t s) {
  if (nsym)
    k_pack<<<blocks_for(nsym, 256, 65536), 256, 0, s>>>(sym, nsym, sym_off, njobs, table, bitpos,
                                                        job_bit0, job_word0, words);
}

// Histogram of the symbols of every job without contended atomics: keys
// (job, symbol) are sorted, and the length of every run of equal keys is
// stored in its bin.
__global__ void k_hist_keys(const uint16_t *sym, size_t nsym, const uint64_t *sym_off, int njobs,
                            uint32_t *keys, uint32_t *idx) {
  for (size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x; s < nsym;
       s += (size_t)gridDim.x * blockDim.x) {
    const int j = job_of_u64(sym_off, njobs, s);
    keys[s] = ((uint32_t)j << 16) | sym[s];
    idx[s] = 0;
  }
}
__global__ void k_run_flags(const uint32_t *keys, size_t nsym, uint8_t *flag) {
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < nsym;
       q += (size_t)gridDim.x * blockDim.x)
    flag[q] = (q == 0 || keys[q] != keys[q - 1]) ? 1 : 0;
}
__global__ void k_run_starts(const uint8_t *flag, const uint32_t *rank, size_t nsym,
                             uint32_t *starts) {
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < nsym;
       q += (size_t)gridDim.x * blockDim.x)
    if (flag[q]) starts[rank[q]] = (uint32_t)q;
}
// run r spans [starts[r], starts[r + 1]); its length is its key's count
__global__ void k_run_hist(const uint32_t *keys, const uint32_t *starts, const uint32_t *nruns,
                           size_t nsym, uint32_t *hist) {
  const uint32_t R = *nruns;
  for (size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x; r < R;
       r += (size_t)gridDim.x * blockDim.x) {
    const uint32_t s = starts[r];
    const uint32_t e = r + 1 < R ? starts[r + 1] : (uint32_t)nsym;
    const uint32_t k = keys[s];
    hist[(size_t)(k >> 16) * 65536 + (k & 0xffffu)] = e - s;
  }
}

void symbol_histogram(const uint16_t *sym, size_t nsym, const uint64_t *sym_off, int njobs,
                      uint32_t *hist, Arena &ar, hipStream_t s) {
  fill_u32(hist, 0, (size_t)njobs * 65536, s);
  if (!nsym) return;
  if (nsym > 0xffffffffull) throw Error(-6, "more than 2^32 - 1 edit symbols");
  uint32_t *keys = ar.get<uint32_t>(nsym), *idx = ar.get<uint32_t>(nsym);
  uint8_t *flag = ar.get<uint8_t>(nsym);
  uint32_t *rank = ar.get<uint32_t>(nsym), *starts = ar.get<uint32_t>(nsym);
  uint32_t *nruns = ar.get<uint32_t>(1);
  const int nb = blocks_for(nsym, 256, 65536);
  k_hist_keys<<<nb, 256, 0, s>>>(sym, nsym, sym_off, njobs, keys, idx);
  int jb = 0;
  while (jb < 16 && ((uint32_t)(njobs - 1) >> jb) != 0) ++jb;
  radix_sort_u32(keys, idx, nsym, 16 + jb, ar, s);
  k_run_flags<<<nb, 256, 0, s>>>(keys, nsym, flag);
  scan_u8_u32(flag, rank, nsym, nruns, ar, s);
  k_run_starts<<<nb, 256, 0, s>>>(flag, rank, nsym, starts);
  k_run_hist<<<nb, 256, 0, s>>>(keys, starts, nruns, nsym, hist);
}

// float64 coordinates before quantisation, in each job's particle order
__global__ void k_debug_rec(EncBufs B) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < B.n;
       k += (size_t)gridDim.x * blockDim.x) {
    const int j = job_of(B.p_off, B.njobs, (int64_t)k);
    const int64_t g = B.p_off[j] + __float_as_uint(B.pos[k].w);
    const float4 r = B.rec[k];
    B.debug[g] = (double)r.x;
    B.debug[B.n + g] = (double)r.y;
    B.debug[2 * B.n + g] = (double)r.z;
  }
}
__global__ void k_debug_e(EncBufs B) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < B.ne;
       e += (size_t)gridDim.x * blockDim.x) {
    const int j = job_of(B.e_off, B.njobs, (int64_t)e);
    const uint32_t k = B.e_list[e];
    const int64_t g = B.p_off[j] + __float_as_uint(B.pos[k].w);
    const double3 p = final_pos(B, j, e);
    B.debug[g] = p.x;
    B.debug[B.n + g] = p.y;
    B.debug[2 * B.n + g] = p.z;
  }
}

void launch_debug_xyz(const EncBufs &b, hipStream_t s) {
  if (b.n) k_debug_rec<<<blocks_for(b.n, 256, 65536), 256, 0, s>>>(b);
  if (b.ne) k_debug_e<<<blocks_for(b.ne, 256, 65536), 256, 0, s>>>(b);
}

}  // namespace pcc
