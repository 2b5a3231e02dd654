// Host half of the edit stream (Sec. 3.3: Huffman coding followed by ZSTD):
// length-limited canonical Huffman tables from the device histograms, ZSTD
// through the system runtime library (opened with dlopen; the stream is
// stored uncompressed when it is missing), stream assembly and decoding.
//
// Byte layout (little-endian):
//   header, 64 bytes: u32 magic 0x45434350 | u16 version 2 | u8 m | u8 flags
//     (bit 0: payload is one ZSTD frame, bit 1: Huffman-coded symbols)
//     | u64 n | u64 flagged | f64 step | f64 offset | u64 raw payload bytes
//     | u64 stored payload bytes | u32 symbol bits (8 or 16) | u32 0
//   payload: ceil(n/8) flag bytes (particle k at bit k mod 8 of byte k / 8),
//     then for flagged > 0: u32 K | K u32 symbols | K u8 code lengths |
//     u64 bit count | u32 C | u32 0 | the u64 stream bit at which each chunk
//     of C symbols starts (the last chunk may be shorter) | the bits; the
//     chunk starts let the device decoder give every chunk its own thread.
//     Symbols run x plane, y plane, z plane, each
//     over the flagged particles in increasing index; m = 32 codes are a low
//     then a high 16-bit symbol.  Canonical codes in (length, symbol) order,
//     most significant bit first; stream bit q is bit q mod 8 of byte q / 8.
//   decoding: edit = code * step - offset; x' = float32(x_hat + edit).
#include <dlfcn.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <queue>
#include <thread>

#include "host.hpp"

namespace pcc {

namespace {
constexpr uint32_t kMagic = 0x45434350u;
constexpr uint16_t kVersion = 2;
constexpr int kMaxLen = 24;
constexpr size_t kHeader = 64;

struct Zstd {
  bool ok = false;
  size_t (*bound)(size_t) = nullptr;
  size_t (*compress)(void *, size_t, const void *, size_t, int) = nullptr;
  size_t (*decompress)(void *, size_t, const void *, size_t) = nullptr;
  unsigned (*is_error)(size_t) = nullptr;
};

Zstd &zstd() {
  static Zstd z;
  static std::once_flag once;
  std::call_once(once, [] {
    void *h = dlopen("libzstd.so.1", RTLD_NOW | RTLD_LOCAL);
    if (!h) return;
    z.bound = (size_t(*)(size_t))dlsym(h, "ZSTD_compressBound");
    z.compress = (size_t(*)(void *, size_t, const void *, size_t, int))dlsym(h, "ZSTD_compress");
    z.decompress = (size_t(*)(void *, size_t, const void *, size_t))dlsym(h, "ZSTD_decompress");
    z.is_error = (unsigned (*)(size_t))dlsym(h, "ZSTD_isError");
    z.ok = z.bound && z.compress && z.decompress && z.is_error;
  });
  return z;
}

// inputs from this size on are split into pieces of at least this size
constexpr size_t kZstdParallelMin = (size_t)1 << 20;
constexpr size_t kZstdJob = (size_t)512 << 10;
// ZSTD level of the stream payload: the payload is mostly Huffman output and
// a sparse flag mask, for which the fastest level loses little
constexpr int kZstdLevelDefault = 1;

template <typename T>
void put(std::vector<uint8_t> &b, size_t at, T v) {
  std::memcpy(b.data() + at, &v, sizeof v);
}
template <typename T>
T get(const uint8_t *p) {
  T v;
  std::memcpy(&v, p, sizeof v);
  return v;
}

uint32_t reverse_bits(uint32_t c, int len) {
  uint32_t r = 0;
  for (int k = 0; k < len; ++k) r |= ((c >> k) & 1u) << (len - 1 - k);
  return r;
}
}  // namespace

bool zstd_available() { return zstd().ok; }

// Inputs from kZstdParallelMin on are cut into pieces compressed on host
// threads as independent frames; the frames are concatenated, which one
// ZSTD decompression call reads back as a whole.  The input is a list of
// segments (the payload's parts where they already are), so the payload is
// never assembled in one buffer; frames are written after `at` bytes of dst.
struct Segment {
  const uint8_t *p;
  size_t n;
};
static bool zstd_compress_segments(const std::vector<Segment> &segs, size_t at,
                                   std::vector<uint8_t> &dst, int level) {
  Zstd &z = zstd();
  if (!z.ok) return false;
  // the pieces: each segment cut into runs of at most kZstdJob bytes once
  // the payload reaches kZstdParallelMin
  size_t len = 0;
  for (const Segment &g : segs) len += g.n;
  if (len == 0) return false;
  std::vector<Segment> pieces;
  const size_t cut = len >= kZstdParallelMin ? kZstdJob : len;
  for (const Segment &g : segs)
    for (size_t a = 0; a < g.n; a += cut) pieces.push_back({g.p + a, std::min(cut, g.n - a)});
  const size_t np = pieces.size();
  std::vector<std::vector<uint8_t>> out(np);
  std::vector<size_t> got(np, 0);
  std::atomic<size_t> next{0};
  auto work = [&]() {
    for (size_t p; (p = next.fetch_add(1)) < np;) {
      out[p].resize(z.bound(pieces[p].n));
      got[p] = z.compress(out[p].data(), out[p].size(), pieces[p].p, pieces[p].n, level);
    }
  };
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const size_t nth = std::min<size_t>(std::min<size_t>(16, hw), np);
  std::vector<std::thread> th;
  for (size_t t = 1; t < nth; ++t) th.emplace_back(work);
  work();
  for (auto &t : th) t.join();
  size_t total = 0;
  for (size_t p = 0; p < np; ++p) {
    if (z.is_error(got[p])) return false;
    total += got[p];
  }
  dst.resize(at + total);
  for (size_t p = 0; p < np; ++p) {
    std::memcpy(dst.data() + at, out[p].data(), got[p]);
    at += got[p];
  }
  return true;
}

bool zstd_compress(const uint8_t *src, size_t len, std::vector<uint8_t> &dst, int level) {
  dst.clear();
  return zstd_compress_segments({{src, len}}, 0, dst, level);
}

bool zstd_decompress(const uint8_t *src, size_t len, uint8_t *dst, size_t raw_len) {
  Zstd &z = zstd();
  if (!z.ok) return false;
  size_t got = z.decompress(dst, raw_len, src, len);
  return !z.is_error(got) && got == raw_len;
}

// Huffman code lengths by repeatedly merging the two lightest trees (binary
// heap, ties broken by node number); if a code would exceed 24 bits the
// counts are halved and the tree is rebuilt.
void huffman_build(const uint32_t *hist, int alphabet, HuffTable &out) {
  out.syms.clear();
  out.lens.clear();
  out.table.assign(65536, 0);
  std::vector<uint64_t> w;
  for (int s = 0; s < alphabet; ++s)
    if (hist[s]) {
      out.syms.push_back((uint32_t)s);
      w.push_back(hist[s]);
    }
  const size_t k = out.syms.size();
  if (k == 0) return;
  std::vector<uint8_t> len(k, 1);
  if (k > 1) {
    for (;;) {
      using Item = std::pair<uint64_t, uint32_t>;
      std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
      std::vector<uint32_t> parent(2 * k - 1, 0);
      for (size_t i = 0; i < k; ++i) heap.push({w[i], (uint32_t)i});
      uint32_t next = (uint32_t)k;
      while (heap.size() > 1) {
        Item a = heap.top();
        heap.pop();
        Item b = heap.top();
        heap.pop();
        parent[a.second] = next;
        parent[b.second] = next;
        heap.push({a.first + b.first, next});
        ++next;
      }
      std::vector<int> depth(2 * k - 1, 0);
      int deepest = 0;
      for (int id = (int)(2 * k - 3); id >= 0; --id) {
        depth[id] = depth[parent[id]] + 1;
        if (id < (int)k) deepest = std::max(deepest, depth[id]);
      }
      if (deepest <= kMaxLen) {
        for (size_t i = 0; i < k; ++i) len[i] = (uint8_t)depth[i];
        break;
      }
      for (auto &x : w) x = (x + 1) / 2;
    }
  }
  std::vector<uint32_t> order(k);
  for (size_t i = 0; i < k; ++i) order[i] = (uint32_t)i;
  std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
    return len[a] != len[b] ? len[a] < len[b] : out.syms[a] < out.syms[b];
  });
  std::vector<uint32_t> syms(k);
  std::vector<uint8_t> lens(k);
  uint32_t code = 0;
  for (size_t r = 0; r < k; ++r) {
    const uint32_t i = order[r];
    if (r > 0) code = (code + 1) << (len[i] - lens[r - 1]);
    syms[r] = out.syms[i];
    lens[r] = len[i];
    out.table[syms[r]] = reverse_bits(code, len[i]) | ((uint32_t)len[i] << 24);
  }
  out.syms.swap(syms);
  out.lens.swap(lens);
}

size_t stream_bound(int64_t n, int m_bits) {
  if (n < 0) n = 0;
  const size_t per = m_bits == 32 ? 2 : 1;
  const size_t nsym = (size_t)n * 3 * per;
  const size_t raw = ((size_t)n + 7) / 8 + 4 + 5 * 65536 + 8 + 8 +
                     8 * ((nsym + kHuffChunk - 1) / kHuffChunk) + (nsym * kMaxLen + 7) / 8;
  return kHeader + raw + raw / 128 + 4096;
}

void assemble_stream(int64_t n, int m_bits, int64_t nflagged, double qstep, double qoffset,
                     const uint8_t *flags, size_t nflag_bytes, const HuffTable *ht,
                     const uint32_t *words, uint64_t nbits, const uint64_t *chunk_bits,
                     size_t nchunks, std::vector<uint8_t> &out, size_t *payload_raw) {
  const size_t nb = ((size_t)n + 7) / 8;
  const bool huff = nflagged > 0 && ht && !ht->syms.empty();
  const size_t nsym = (size_t)nflagged * 3 * (m_bits == 32 ? 2 : 1);
  if (huff && nchunks != (nsym + kHuffChunk - 1) / kHuffChunk)
    throw Error(PCC_E_DEVICE, "chunk index does not match the symbol count");
  // the payload's parts: flag bytes, the code table and chunk index, the bits
  std::vector<uint8_t> flag_tail;  // flag bytes the caller did not supply
  if (nflag_bytes < nb) flag_tail.assign(nb - nflag_bytes, 0);
  std::vector<uint8_t> tab;
  if (huff) {
    tab.assign(4 + 5 * ht->syms.size() + 8 + 8 + 8 * nchunks, 0);
    size_t at = 0;
    put<uint32_t>(tab, at, (uint32_t)ht->syms.size());
    at += 4;
    for (uint32_t sy : ht->syms) {
      put<uint32_t>(tab, at, sy);
      at += 4;
    }
    for (uint8_t l : ht->lens) tab[at++] = l;
    put<uint64_t>(tab, at, nbits);
    at += 8;
    put<uint32_t>(tab, at, kHuffChunk);
    at += 8;
    for (size_t c = 0; c < nchunks; ++c, at += 8) put<uint64_t>(tab, at, chunk_bits[c]);
  }
  std::vector<Segment> segs;
  if (nb) segs.push_back({flags, std::min(nb, nflag_bytes)});
  if (!flag_tail.empty()) segs.push_back({flag_tail.data(), flag_tail.size()});
  if (huff) {
    segs.push_back({tab.data(), tab.size()});
    segs.push_back({reinterpret_cast<const uint8_t *>(words), (size_t)((nbits + 7) / 8)});
  }
  size_t raw = 0;
  for (const Segment &g : segs) raw += g.n;
  *payload_raw = raw;
  const bool zok = zstd_compress_segments(segs, kHeader, out, kZstdLevelDefault);
  if (!zok) {
    out.assign(kHeader + raw, 0);
    size_t at = kHeader;
    for (const Segment &g : segs) {
      if (g.n) std::memcpy(out.data() + at, g.p, g.n);
      at += g.n;
    }
  }
  const size_t stored = out.size() - kHeader;
  put<uint32_t>(out, 0, kMagic);
  put<uint16_t>(out, 4, kVersion);
  out[6] = (uint8_t)m_bits;
  out[7] = (uint8_t)((zok ? 1 : 0) | (huff ? 2 : 0));
  put<uint64_t>(out, 8, (uint64_t)n);
  put<uint64_t>(out, 16, (uint64_t)nflagged);
  put<double>(out, 24, qstep);
  put<double>(out, 32, qoffset);
  put<uint64_t>(out, 40, (uint64_t)raw);
  put<uint64_t>(out, 48, (uint64_t)stored);
  put<uint32_t>(out, 56, (uint32_t)(m_bits == 8 ? 8 : 16));
  put<uint32_t>(out, 60, 0u);
}

pcc_status parse_stream(const uint8_t *s, size_t len, int64_t n, ParsedStream &out,
                        std::string &err, bool huffman_on_host) {
  if (len < kHeader || get<uint32_t>(s) != kMagic)
    return err = "not an edit stream", PCC_E_INVALID_ARG;
  if (get<uint16_t>(s + 4) != kVersion)
    return err = "edit stream of another format version", PCC_E_INVALID_ARG;
  const int m = s[6], fl = s[7];
  if ((int64_t)get<uint64_t>(s + 8) != n) return err = "particle count differs from the stream", PCC_E_INVALID_ARG;
  const uint64_t nf = get<uint64_t>(s + 16);
  const double step = get<double>(s + 24), offset = get<double>(s + 32);
  const uint64_t raw = get<uint64_t>(s + 40), stored = get<uint64_t>(s + 48);
  const uint32_t symbits = get<uint32_t>(s + 56);
  if (stored != len - kHeader || !(m == 8 || m == 16 || m == 32) || !(symbits == 8 || symbits == 16) ||
      nf > (uint64_t)n)
    return err = "corrupt stream header", PCC_E_INVALID_ARG;
  std::vector<uint8_t> &pay = out.payload;
  pay.assign(raw, 0);
  if (fl & 1) {
    if (!zstd_available()) return err = "stream needs libzstd.so.1", PCC_E_UNSUPPORTED;
    if (!zstd_decompress(s + kHeader, stored, pay.data(), raw)) return err = "ZSTD frame is corrupt", PCC_E_INVALID_ARG;
  } else {
    if (raw != stored) return err = "corrupt stream header", PCC_E_INVALID_ARG;
    if (raw) std::memcpy(pay.data(), s + kHeader, raw);
  }
  const size_t nb = ((size_t)n + 7) / 8;
  if (raw < nb) return err = "payload too short", PCC_E_INVALID_ARG;
  const int per = m == 32 ? 2 : 1;
  const size_t nsym = (size_t)nf * 3 * per;
  std::vector<uint32_t> &sym = out.sym;
  sym.assign((fl & 2) && !huffman_on_host ? 0 : nsym, 0);
  const uint8_t *p = pay.data() + nb, *end = pay.data() + raw;
  if (nsym && (fl & 2)) {
    if (end - p < 4) return err = "payload too short", PCC_E_INVALID_ARG;
    const uint32_t k = get<uint32_t>(p);
    p += 4;
    if ((size_t)(end - p) < (size_t)k * 5 + 8) return err = "payload too short", PCC_E_INVALID_ARG;
    std::vector<uint32_t> syms(k);
    std::vector<int> count(kMaxLen + 1, 0);
    for (uint32_t i = 0; i < k; ++i) syms[i] = get<uint32_t>(p + 4 * i);
    p += 4 * (size_t)k;
    std::vector<uint8_t> lens(p, p + k);
    p += k;
    const uint64_t nbits = get<uint64_t>(p);
    p += 8;
    if (end - p < 8) return err = "payload too short", PCC_E_INVALID_ARG;
    const uint32_t chunk = get<uint32_t>(p);
    p += 8;
    if (chunk == 0) return err = "corrupt chunk index", PCC_E_INVALID_ARG;
    const size_t nchunks = (nsym + chunk - 1) / chunk;
    if ((size_t)(end - p) / 8 < nchunks) return err = "payload too short", PCC_E_INVALID_ARG;
    const uint8_t *index = p;
    p += 8 * nchunks;
    if ((uint64_t)(end - p) * 8 < nbits) return err = "payload too short", PCC_E_INVALID_ARG;
    // chunk starts: from bit 0, non-decreasing, inside the bitstream
    for (size_t c = 0; c < nchunks; ++c) {
      const uint64_t b = get<uint64_t>(index + 8 * c);
      if ((c == 0 && b != 0) || (c > 0 && b < get<uint64_t>(index + 8 * (c - 1))) || b > nbits)
        return err = "corrupt chunk index", PCC_E_INVALID_ARG;
    }
    // symbols in canonical order: by length, then symbol value
    std::vector<uint32_t> order(k);
    for (uint32_t i = 0; i < k; ++i) {
      if (lens[i] == 0 || lens[i] > kMaxLen) return err = "bad code length", PCC_E_INVALID_ARG;
      order[i] = i;
      count[lens[i]]++;
    }
    std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
      return lens[a] != lens[b] ? lens[a] < lens[b] : syms[a] < syms[b];
    });
    out.huff = true;
    out.canon_sym.resize(k);
    out.canon_len.resize(k);
    for (uint32_t r = 0; r < k; ++r) {
      out.canon_sym[r] = syms[order[r]];
      out.canon_len[r] = lens[order[r]];
    }
    out.nbits = nbits;
    out.chunk = chunk;
    out.nchunks = nchunks;
    out.index_at = (size_t)(index - pay.data());
    out.bits_at = (size_t)(p - pay.data());
    uint64_t q = 0;
    for (size_t t = 0; huffman_on_host && t < nsym; ++t) {
      if (t % chunk == 0 && get<uint64_t>(index + 8 * (t / chunk)) != q)
        return err = "corrupt chunk index", PCC_E_INVALID_ARG;
      // walk the code lengths: codes of length l are a contiguous range
      int64_t code = 0, first = 0, index = 0;
      int l = 1;
      for (;; ++l) {
        if (l > kMaxLen || q >= nbits) return err = "corrupt Huffman data", PCC_E_INVALID_ARG;
        code |= (p[q >> 3] >> (q & 7)) & 1;
        ++q;
        const int64_t c = count[l];
        if (code - first < c) {
          sym[t] = syms[order[index + (code - first)]];
          break;
        }
        index += c;
        first = (first + c) << 1;
        code <<= 1;
      }
    }
  } else if (nsym) {
    const size_t bytes = symbits / 8;
    if ((size_t)(end - p) < nsym * bytes) return err = "payload too short", PCC_E_INVALID_ARG;
    for (size_t t = 0; t < nsym; ++t) {
      uint32_t v = 0;
      for (size_t b = 0; b < bytes; ++b) v |= (uint32_t)p[bytes * t + b] << (8 * b);
      sym[t] = v;
    }
  }
  out.n = n;
  out.nflagged = nf;
  out.per = per;
  out.step = step;
  out.offset = offset;
  out.flag_bytes = nb;
  // the flag count must match the header
  uint64_t cnt = 0;
  for (size_t b = 0; b < nb; ++b) cnt += (uint64_t)__builtin_popcount(pay[b]);
  if (n % 8 && nb) cnt -= (uint64_t)__builtin_popcount(pay[nb - 1] >> (n % 8));
  if (cnt != nf) return err = "flag count differs from the header", PCC_E_INVALID_ARG;
  return PCC_OK;
}

pcc_status decode_stream(const uint8_t *s, size_t len, int64_t n, const float *rx, const float *ry,
                         const float *rz, float *ox, float *oy, float *oz, std::string &err) {
  ParsedStream ps;
  const pcc_status st = parse_stream(s, len, n, ps, err, true);
  if (st != PCC_OK) return st;
  const std::vector<uint8_t> &pay = ps.payload;
  const std::vector<uint32_t> &sym = ps.sym;
  const uint64_t nf = ps.nflagged;
  const int per = ps.per;
  const double step = ps.step, offset = ps.offset;
  const float *rin[3] = {rx, ry, rz};
  float *rout[3] = {ox, oy, oz};
  for (int a = 0; a < 3; ++a)
    if (n) std::memcpy(rout[a], rin[a], (size_t)n * sizeof(float));
  // flagged particle ids in increasing order
  std::vector<int64_t> ids;
  ids.reserve(nf);
  for (int64_t k = 0; k < n; ++k)
    if ((pay[k >> 3] >> (k & 7)) & 1) ids.push_back(k);
  for (int a = 0; a < 3; ++a)
    for (size_t r = 0; r < ids.size(); ++r) {
      const size_t base = ((size_t)a * nf + r) * per;
      const uint64_t code = per == 2 ? ((uint64_t)sym[base] | ((uint64_t)sym[base + 1] << 16)) : sym[base];
      const double edit = (double)code * step - offset;
      rout[a][ids[r]] = (float)((double)rin[a][ids[r]] + edit);
    }
  return PCC_OK;
}

}  // namespace pcc
