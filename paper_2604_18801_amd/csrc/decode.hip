// Edit application on the device (Sec. 3.3, reconstruction of the edited
// data).  The host undoes ZSTD and reads the stream's tables (flag mask,
// the canonical Huffman code, the chunk index); the Huffman bitstream is
// decoded on the device, one thread per chunk of symbols starting at the
// bit the chunk index gives; a scan ranks the flagged particles and one
// kernel writes x' = float32(x_hat + code * s - 2 xi) for flagged particles
// and x_hat for the others, with the host decoder's arithmetic (float64, no
// contraction), so both give the same bits.
#include <cstring>
#include <vector>

#include "host.hpp"

namespace pcc {

__global__ void k_flag_popc(const uint8_t *flags, size_t nb, uint8_t *popc) {
  for (size_t b = (size_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb;
       b += (size_t)gridDim.x * blockDim.x)
    popc[b] = (uint8_t)__popc((uint32_t)flags[b]);
}

__global__ void k_apply_edits(const uint8_t *flags, const uint32_t *byte_rank, const uint32_t *sym,
                              uint64_t nf, int per, double step, double offset, int64_t n,
                              const float *rx, const float *ry, const float *rz, float *ox,
                              float *oy, float *oz) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t byte = flags[k >> 3], bit = (uint32_t)(k & 7);
    float x = rx[k], y = ry[k], z = rz[k];
    if ((byte >> bit) & 1u) {
      const uint64_t r = byte_rank[k >> 3] + (uint32_t)__popc(byte & ((1u << bit) - 1u));
      double v[3] = {(double)x, (double)y, (double)z};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const size_t base = ((size_t)a * nf + r) * per;
        const uint64_t code =
            per == 2 ? ((uint64_t)sym[base] | ((uint64_t)sym[base + 1] << 16)) : sym[base];
        const double edit = (double)code * step - offset;
        v[a] = v[a] + edit;
      }
      x = (float)v[0];
      y = (float)v[1];
      z = (float)v[2];
    }
    ox[k] = x;
    oy[k] = y;
    oz[k] = z;
  }
}

// Canonical Huffman decoding.  Codes of at most kLutBits bits come from a
// table indexed by the next kLutBits stream bits (entry: canonical index << 5
// | length, 0 for a longer code); longer codes are found by length, codes of
// one length being a contiguous range from first[l] (canonical index
// base[l] on).
constexpr int kLutBits = 11;
constexpr int kHuffMaxLen = 24;

struct HuffDec {
  const uint32_t *words;   // the bitstream as little-endian words, 3 zero words after it
  const uint64_t *start;   // first stream bit of each chunk
  const uint32_t *lut;     // [1 << kLutBits]
  const uint32_t *canon;   // symbol of each canonical index
  uint32_t *sym;           // decoded symbols
  uint32_t *err;           // set when the bitstream is corrupt
  uint64_t nbits, nsym, nchunks;
  uint32_t chunk;
  uint32_t first[kHuffMaxLen + 1], count[kHuffMaxLen + 1], base[kHuffMaxLen + 1];
};

__global__ void __launch_bounds__(256) k_huff_decode(HuffDec H) {
  __shared__ uint32_t lut[1 << kLutBits];
  for (int i = threadIdx.x; i < (1 << kLutBits); i += blockDim.x) lut[i] = H.lut[i];
  __syncthreads();
  for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < H.nchunks;
       c += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t pos = H.start[c];
    const uint64_t end = c + 1 < H.nchunks ? H.start[c + 1] : H.nbits;
    const uint64_t s0 = c * H.chunk, s1 = s0 + H.chunk < H.nsym ? s0 + H.chunk : H.nsym;
    if (pos > end) {
      atomicOr(H.err, 1u);
      continue;
    }
    // a window of three words over the stream: w0 holds bit pos
    uint64_t wi = pos >> 5;
    uint32_t w0 = H.words[wi], w1 = H.words[wi + 1], w2 = H.words[wi + 2];
    bool bad = false;
    for (uint64_t t = s0; t < s1; ++t) {
      const uint32_t sh = (uint32_t)(pos - (wi << 5));
      const uint64_t x = ((uint64_t)w1 << 32) | w0;
      // the next 32 stream bits, the first one at the top
      const uint32_t v = __builtin_bitreverse32((uint32_t)(x >> sh));
      const uint32_t e = lut[v >> (32 - kLutBits)];
      uint32_t len = e & 31u, idx = e >> 5;
      if (len == 0) {
        for (int l = kLutBits + 1; l <= kHuffMaxLen; ++l) {
          const uint32_t code = v >> (32 - l);
          if (code - H.first[l] < H.count[l]) {
            idx = H.base[l] + (code - H.first[l]);
            len = (uint32_t)l;
            break;
          }
        }
        if (len == 0) {
          bad = true;
          break;
        }
      }
      H.sym[t] = H.canon[idx];
      pos += len;
      if (pos > end) {  // (also keeps the window inside the stream)
        bad = true;
        break;
      }
      if (pos - (wi << 5) >= 32) {
        ++wi;
        w0 = w1;
        w1 = w2;
        w2 = H.words[wi + 2];
      }
    }
    if (bad || pos != end) atomicOr(H.err, 1u);
  }
}

bool apply_edits_device(const ParsedStream &ps, const float *const rin[3], float *const rout[3],
                        Arena &ar, hipStream_t s) {
  const int64_t n = ps.n;
  if (n <= 0) return true;
  const size_t nb = ps.flag_bytes;
  uint8_t *flags = ar.get<uint8_t>(nb);
  uint8_t *popc = ar.get<uint8_t>(nb);
  uint32_t *rank = ar.get<uint32_t>(nb);
  uint32_t *tot = ar.get<uint32_t>(1);
  const size_t nsym = (size_t)ps.nflagged * 3 * ps.per;
  uint32_t *sym = ar.get<uint32_t>(nsym ? nsym : 1);
  PCC_HIP(hipMemcpyAsync(flags, ps.payload.data(), nb, hipMemcpyHostToDevice, s));
  if (nsym && ps.huff) {
    // tables of the canonical code
    const size_t k = ps.canon_sym.size();
    HuffDec H;
    std::memset(&H, 0, sizeof H);
    std::vector<uint32_t> lut((size_t)1 << kLutBits, 0u);
    uint32_t code = 0;
    for (size_t r = 0; r < k; ++r) {
      const int l = ps.canon_len[r];
      if (r > 0) code = (code + 1) << (l - ps.canon_len[r - 1]);
      if (code >> l) return false;  // lengths that no prefix code has
      if (H.count[l] == 0) {
        H.first[l] = code;
        H.base[l] = (uint32_t)r;
      }
      H.count[l]++;
      if (l <= kLutBits) {
        const uint32_t lo = code << (kLutBits - l), hi = (code + 1) << (kLutBits - l);
        for (uint32_t i = lo; i < hi; ++i) lut[i] = ((uint32_t)r << 5) | (uint32_t)l;
      }
    }
    const size_t nwords = (size_t)((ps.nbits + 31) / 32) + 3;
    uint32_t *words = ar.get<uint32_t>(nwords);
    uint64_t *start = ar.get<uint64_t>(ps.nchunks);
    uint32_t *d_lut = ar.get<uint32_t>(lut.size());
    uint32_t *canon = ar.get<uint32_t>(k ? k : 1);
    uint32_t *err = ar.get<uint32_t>(1);
    fill_u32(words, 0, nwords, s);
    fill_u32(err, 0, 1, s);
    PCC_HIP(hipMemcpyAsync(words, ps.payload.data() + ps.bits_at, (size_t)((ps.nbits + 7) / 8),
                           hipMemcpyHostToDevice, s));
    PCC_HIP(hipMemcpyAsync(start, ps.payload.data() + ps.index_at, ps.nchunks * sizeof(uint64_t),
                           hipMemcpyHostToDevice, s));
    PCC_HIP(hipMemcpyAsync(d_lut, lut.data(), lut.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    if (k) PCC_HIP(hipMemcpyAsync(canon, ps.canon_sym.data(), k * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    H.words = words;
    H.start = start;
    H.lut = d_lut;
    H.canon = canon;
    H.sym = sym;
    H.err = err;
    H.nbits = ps.nbits;
    H.nsym = nsym;
    H.nchunks = ps.nchunks;
    H.chunk = ps.chunk;
    k_huff_decode<<<blocks_for(ps.nchunks, 256, 4096), 256, 0, s>>>(H);
    uint32_t herr = 0;
    PCC_HIP(hipMemcpyAsync(&herr, err, sizeof herr, hipMemcpyDeviceToHost, s));
    PCC_HIP(hipStreamSynchronize(s));
    if (herr) return false;
  } else if (nsym) {
    PCC_HIP(hipMemcpyAsync(sym, ps.sym.data(), nsym * sizeof(uint32_t), hipMemcpyHostToDevice, s));
  }
  k_flag_popc<<<blocks_for(nb, 256, 65536), 256, 0, s>>>(flags, nb, popc);
  scan_u8_u32(popc, rank, nb, tot, ar, s);
  k_apply_edits<<<blocks_for((size_t)n, 256, 65536), 256, 0, s>>>(
      flags, rank, sym, ps.nflagged, ps.per, ps.step, ps.offset, n, rin[0], rin[1], rin[2],
      rout[0], rout[1], rout[2]);
  // the host buffers above must outlive the copies
  PCC_HIP(hipStreamSynchronize(s));
  return true;
}

}  // namespace pcc
