// Cell build (Sec. 2.4.1 cell linking; Sec. 3.3 cell side >= b + 2 sqrt(3) xi):
// input scan, cell keys of the original positions, gather of the sorted
// structure of arrays, unique cells by boundary detection and the forward
// half-shell of 13 neighbour cells.
#include "kernels.hpp"

#include <cfloat>

namespace pcc {

template <typename T>
__device__ inline T wave_reduce_min(T v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = fminf(v, __shfl_xor(v, d, kWave));
  return v;
}
template <typename T>
__device__ inline T wave_reduce_max(T v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, kWave));
  return v;
}
__device__ inline uint32_t wave_reduce_add(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// One block per tile of one job: extent of the originals, largest magnitude,
// and the count of values that are not finite or break |x_hat - x| <= xi.
__global__ void __launch_bounds__(256)
k_scan_inputs(const Tile *tiles, Soa3 o, Soa3 r, const double *xi_job, ScanPart *parts) {
  __shared__ float smn[3][4], smx[3][4], sab[4];
  __shared__ uint32_t sbb[4], sbv[4];
  const Tile t = tiles[blockIdx.x];
  const double xi = xi_job[t.job];
  float mn[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, mx[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
  float ab = 0.f;
  uint32_t bb = 0, bv = 0;
  for (int64_t g = t.start + threadIdx.x; g < t.end; g += blockDim.x) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float xv = o.a[a][g], rv = r.a[a][g];
      if (!isfinite(xv) || !isfinite(rv)) {
        bv++;
        continue;
      }
      mn[a] = fminf(mn[a], xv);
      mx[a] = fmaxf(mx[a], xv);
      ab = fmaxf(ab, fmaxf(fabsf(xv), fabsf(rv)));
      if (fabs((double)rv - (double)xv) > xi) bb++;
    }
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    mn[a] = wave_reduce_min(mn[a]);
    mx[a] = wave_reduce_max(mx[a]);
  }
  ab = wave_reduce_max(ab);
  bb = wave_reduce_add(bb);
  bv = wave_reduce_add(bv);
  if (lane == 0) {
    for (int a = 0; a < 3; ++a) {
      smn[a][w] = mn[a];
      smx[a][w] = mx[a];
    }
    sab[w] = ab;
    sbb[w] = bb;
    sbv[w] = bv;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    ScanPart p;
    for (int a = 0; a < 3; ++a) {
      p.mn[a] = fminf(fminf(smn[a][0], smn[a][1]), fminf(smn[a][2], smn[a][3]));
      p.mx[a] = fmaxf(fmaxf(smx[a][0], smx[a][1]), fmaxf(smx[a][2], smx[a][3]));
    }
    p.maxabs = fmaxf(fmaxf(sab[0], sab[1]), fmaxf(sab[2], sab[3]));
    p.bad_bound = sbb[0] + sbb[1] + sbb[2] + sbb[3];
    p.bad_value = sbv[0] + sbv[1] + sbv[2] + sbv[3];
    p.job = (uint32_t)t.job;
    parts[blockIdx.x] = p;
  }
}

void launch_scan_inputs(const Tile *tiles, int ntiles, Soa3 o, Soa3 r, const double *xi_job,
                        ScanPart *parts, hipStream_t s) {
  if (ntiles) k_scan_inputs<<<ntiles, 256, 0, s>>>(tiles, o, r, xi_job, parts);
}

// cell coordinate along one axis of the job's grid
__device__ inline int64_t cell_coord(double x, double origin, double inv_w, int nc, bool periodic) {
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

__global__ void k_cell_keys(const JobDev *jobs, const int64_t *p_off, int njobs, Soa3 o, size_t n,
                            uint32_t *keys, uint32_t *vals) {
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (size_t)gridDim.x * blockDim.x) {
    const int j = job_of(p_off, njobs, (int64_t)g);
    const JobDev &J = jobs[j];
    int64_t c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      c[a] = cell_coord((double)o.a[a][g], J.origin[a], J.inv_w[a], J.nc[a], (J.periodic >> a) & 1);
    keys[g] = J.cell_base + (uint32_t)((c[2] * J.nc[1] + c[1]) * J.nc[0] + c[0]);
    vals[g] = (uint32_t)g;
  }
}

void launch_cell_keys(const JobDev *jobs, const int64_t *p_off, int njobs, Soa3 o, size_t n,
                      uint32_t *keys, uint32_t *vals, hipStream_t s) {
  if (n) k_cell_keys<<<blocks_for(n, 256, 65536), 256, 0, s>>>(jobs, p_off, njobs, o, n, keys, vals);
}

// Sorted structure of arrays: xyz and the job-local original index in w.
// Written as a scatter: each input particle is read in order (coalesced
// reads of the six coordinate arrays) and its two records go to its sorted
// slot, rather than six 4-byte gathers per sorted slot.
__global__ void k_inv_perm(const uint32_t *perm, size_t n, uint32_t *inv_perm) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x)
    inv_perm[perm[k]] = (uint32_t)k;
}

__global__ void k_scatter_sorted(const uint32_t *inv_perm, const int64_t *p_off, int njobs, Soa3 o,
                                 Soa3 r, size_t n, float4 *pos, float4 *rec) {
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (size_t)gridDim.x * blockDim.x) {
    const uint32_t k = inv_perm[g];
    const int j = job_of(p_off, njobs, (int64_t)g);
    const uint32_t lid = (uint32_t)((int64_t)g - p_off[j]);
    pos[k] = make_float4(o.a[0][g], o.a[1][g], o.a[2][g], __uint_as_float(lid));
    rec[k] = make_float4(r.a[0][g], r.a[1][g], r.a[2][g], 0.f);
  }
}

void launch_gather(const uint32_t *perm, const int64_t *p_off, int njobs, Soa3 o, Soa3 r, size_t n,
                   float4 *pos, float4 *rec, uint32_t *inv_perm, hipStream_t s) {
  if (!n) return;
  const int nb = blocks_for(n, 256, 65536);
  k_inv_perm<<<nb, 256, 0, s>>>(perm, n, inv_perm);
  k_scatter_sorted<<<nb, 256, 0, s>>>(inv_perm, p_off, njobs, o, r, n, pos, rec);
}

__global__ void k_cell_flags(const uint32_t *keys, size_t n, uint8_t *flag) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x)
    flag[k] = (k == 0 || keys[k] != keys[k - 1]) ? 1 : 0;
}

__global__ void k_cell_starts(const uint32_t *keys, const uint8_t *flag, const uint32_t *cid,
                              size_t n, uint32_t *cell_of, uint32_t *cell_start, uint32_t *cell_key,
                              const uint32_t *n_cells) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x) {
    const uint32_t c = cid[k] + flag[k] - 1u;
    cell_of[k] = c;
    if (flag[k]) {
      cell_start[c] = (uint32_t)k;
      cell_key[c] = keys[k];
    }
    if (k == n - 1) cell_start[*n_cells] = (uint32_t)n;
  }
}

void build_cells(const uint32_t *keys, size_t n, uint32_t *cell_of, uint32_t *cell_start,
                 uint32_t *cell_key, uint32_t *n_cells, Arena &ar, hipStream_t s) {
  if (n == 0) {
    fill_u32(n_cells, 0, 1, s);
    fill_u32(cell_start, 0, 1, s);
    return;
  }
  uint8_t *flag = ar.get<uint8_t>(n);
  uint32_t *cid = ar.get<uint32_t>(n);
  const int nb = blocks_for(n, 256, 65536);
  k_cell_flags<<<nb, 256, 0, s>>>(keys, n, flag);
  scan_u8_u32(flag, cid, n, n_cells, ar, s);
  k_cell_starts<<<nb, 256, 0, s>>>(keys, flag, cid, n, cell_of, cell_start, cell_key, n_cells);
}

// blk[b] = first cell whose key is at least b << shift (a coarse index of
// the sorted keys: a neighbour's search then covers the few cells of one
// block instead of all of them)
__global__ void k_key_blocks(const uint32_t *cell_key, const uint32_t *n_cells, size_t nblk,
                             int shift, uint32_t *blk) {
  const uint32_t U = *n_cells;
  for (size_t b = (size_t)blockIdx.x * blockDim.x + threadIdx.x; b <= nblk;
       b += (size_t)gridDim.x * blockDim.x) {
    const uint64_t want = (uint64_t)b << shift;
    uint32_t a = 0, c = U;
    while (a < c) {
      const uint32_t m = (a + c) >> 1;
      if ((uint64_t)cell_key[m] < want)
        a = m + 1;
      else
        c = m;
    }
    blk[b] = a;
  }
}

// The 13 forward neighbour cells of a cell (x, y, z), grouped into runs of
// consecutive keys: slot 0 is the cell (x + 1, y, z); each of the four rows
// (dy, dz) = (1, 0), (-1, 1), (0, 1), (1, 1) holds the cells x - 1 .. x + 1
// at (y + dy, z + dz), whose keys are consecutive unless the row crosses a
// periodic x face: slot 2g - 1 is the part inside [0, nx), slot 2g the cell
// across the face (x = 0: cell nx - 1; x = nx - 1: cell 0), if any.  The
// cells are sorted by key, so each slot is one range of sorted particles.
__device__ inline int cell_bound(const uint32_t *cell_key, uint32_t U, const uint32_t *blk,
                                 int shift, uint64_t key) {
  // first cell whose key is at least `key` (key <= the key space)
  uint32_t a = blk[key >> shift], b = blk[(key >> shift) + 1];
  if (b > U) b = U;
  while (a < b) {
    const uint32_t m = (a + b) >> 1;
    if ((uint64_t)cell_key[m] < key)
      a = m + 1;
    else
      b = m;
  }
  return (int)a;
}

// One thread per (cell, slot).  The thread of slot 0 also records the
// cell's periodic faces: bit 2a when the cell is the first along periodic
// axis a, bit 2a + 1 when it is the last (only for jobs whose coordinates
// lie in their periodic box, where a neighbour cell across a face stands for
// one periodic image).
__global__ void k_neighbor_ranges(const JobDev *jobs, const uint32_t *cell_base, int njobs,
                                  const uint32_t *cell_key, const uint32_t *n_cells,
                                  const uint32_t *cell_start, const uint32_t *blk, int shift,
                                  uint2 *nrange, uint8_t *edge) {
  const uint32_t U = *n_cells;
  const size_t total = (size_t)U * kNbrSlots;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (size_t)gridDim.x * blockDim.x) {
    const size_t u = t / kNbrSlots;
    const int slot = (int)(t - u * kNbrSlots);
    const uint32_t key = cell_key[u];
    // job whose key range holds this cell
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (cell_base[mid] <= key)
        lo = mid;
      else
        hi = mid - 1;
    }
    const JobDev &J = jobs[lo];
    const uint32_t local = key - J.cell_base;
    const int64_t nx = J.nc[0], ny = J.nc[1], nz = J.nc[2];
    const int64_t c[3] = {(int64_t)(local % (uint32_t)nx),
                          (int64_t)((local / (uint32_t)nx) % (uint32_t)ny),
                          (int64_t)(local / ((uint32_t)nx * (uint32_t)ny))};
    if (slot == 0) {
      uint32_t eb = 0;
      if (J.img)
        for (int a = 0; a < 3; ++a)
          if (((J.periodic >> a) & 1) && J.nc[a] >= 3) {
            if (c[a] == 0) eb |= 1u << (2 * a);
            if (c[a] == J.nc[a] - 1) eb |= 1u << (2 * a + 1);
          }
      edge[u] = (uint8_t)eb;
    }
    const bool px = (J.periodic & 1) && nx >= 3;
    int dy = 0, dz = 0;
    int64_t x0, x1;  // the slot's cells x0 .. x1 (empty when x0 > x1)
    if (slot == 0) {
      if (c[0] + 1 < nx) {
        x0 = x1 = c[0] + 1;
      } else if (px) {
        x0 = x1 = 0;
      } else {  // the last cell of an open axis has no x + 1
        x0 = 1;
        x1 = 0;
      }
    } else {
      const int g = (slot - 1) >> 1;
      dy = g == 0 ? 1 : (g == 1 ? -1 : (g == 2 ? 0 : 1));
      dz = g == 0 ? 0 : 1;
      if (slot & 1) {
        x0 = c[0] > 0 ? c[0] - 1 : 0;
        x1 = c[0] + 1 < nx ? c[0] + 1 : nx - 1;
      } else if (px && c[0] == 0) {
        x0 = x1 = nx - 1;
      } else if (px && c[0] == nx - 1) {
        x0 = x1 = 0;
      } else {
        x0 = 1;
        x1 = 0;
      }
    }
    int64_t y = c[1] + dy, z = c[2] + dz;
    bool ok = x0 <= x1;
    if (y < 0 || y >= ny) {
      if ((J.periodic & 2) && ny >= 3)
        y = (y + ny) % ny;
      else
        ok = false;
    }
    if (z < 0 || z >= nz) {
      if ((J.periodic & 4) && nz >= 3)
        z = (z + nz) % nz;
      else
        ok = false;
    }
    uint2 r = make_uint2(0u, 0u);
    if (ok) {
      const uint64_t row = (uint64_t)J.cell_base + (uint64_t)((z * ny + y) * nx);
      const int a = cell_bound(cell_key, U, blk, shift, row + (uint64_t)x0);
      const int b = cell_bound(cell_key, U, blk, shift, row + (uint64_t)x1 + 1);
      r = make_uint2(cell_start[a], cell_start[b]);
    }
    nrange[t] = r;
  }
}

void launch_neighbors(const JobDev *jobs, const uint32_t *cell_base, int njobs,
                      const uint32_t *cell_key, const uint32_t *n_cells, const uint32_t *cell_start,
                      size_t max_cells, uint64_t key_space, uint2 *nrange, uint8_t *edge,
                      Arena &ar, hipStream_t s) {
  if (!max_cells) return;
  // about four keys' blocks per particle at most
  int shift = 0;
  while ((key_space >> shift) > max_cells / 4 + 1) ++shift;
  const size_t nblk = (size_t)(key_space >> shift) + 1;
  uint32_t *blk = ar.get<uint32_t>(nblk + 1);
  k_key_blocks<<<blocks_for(nblk + 1, 256, 65536), 256, 0, s>>>(cell_key, n_cells, nblk, shift, blk);
  k_neighbor_ranges<<<blocks_for(max_cells * kNbrSlots, 256, 65536), 256, 0, s>>>(
      jobs, cell_base, njobs, cell_key, n_cells, cell_start, blk, shift, nrange, edge);
}

}  // namespace pcc
