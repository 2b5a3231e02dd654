// Edit application on the device (Sec. 3.3, reconstruction of the edited
// data): the host parses the stream (ZSTD, then the sequential Huffman
// bitstream) into the flag mask and the code planes; a scan ranks the
// flagged particles and one kernel writes x' = float32(x_hat + code * s -
// 2 xi) for flagged particles and x_hat for the others, with the host
// decoder's arithmetic (float64, no contraction), so both give the same bits.
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

void apply_edits_device(const ParsedStream &ps, const float *const rin[3], float *const rout[3],
                        Arena &ar, hipStream_t s) {
  const int64_t n = ps.n;
  if (n <= 0) return;
  const size_t nb = ps.flag_bytes;
  uint8_t *flags = ar.get<uint8_t>(nb);
  uint8_t *popc = ar.get<uint8_t>(nb);
  uint32_t *rank = ar.get<uint32_t>(nb);
  uint32_t *tot = ar.get<uint32_t>(1);
  const size_t nsym = ps.sym.size();
  uint32_t *sym = ar.get<uint32_t>(nsym ? nsym : 1);
  PCC_HIP(hipMemcpyAsync(flags, ps.payload.data(), nb, hipMemcpyHostToDevice, s));
  if (nsym) PCC_HIP(hipMemcpyAsync(sym, ps.sym.data(), nsym * sizeof(uint32_t), hipMemcpyHostToDevice, s));
  k_flag_popc<<<blocks_for(nb, 256, 65536), 256, 0, s>>>(flags, nb, popc);
  scan_u8_u32(popc, rank, nb, tot, ar, s);
  k_apply_edits<<<blocks_for((size_t)n, 256, 65536), 256, 0, s>>>(
      flags, rank, sym, ps.nflagged, ps.per, ps.step, ps.offset, n, rin[0], rin[1], rin[2],
      rout[0], rout[1], rout[2]);
  // the host buffers above must outlive the copies
  PCC_HIP(hipStreamSynchronize(s));
}

}  // namespace pcc
