// k_sort.hip -- counting sort of parcels by grid-box tile: tile key, rank
// inside the tile and histogram in one pass, exclusive scan of the
// histogram, then an atomic-free scatter of the whole parcel state into the
// second buffer set at offset[key] + rank.  Parcels that are already nearly
// sorted share keys across a wavefront, so the histogram counter of a key
// is bumped once per run of equal keys within a wave.
#include "mpt_internal.h"

namespace mpt {

constexpr int kScanChunk = 1024;   // entries per scan block (256 threads x 4)

// For lanes holding `key` (valid lanes form a prefix of the wave), add the
// length of each run of equal keys to the key's counter *ctr once and
// return, for every lane, the old counter value plus the lane's rank inside
// its run.
__device__ __forceinline__ uint32_t wave_run_add(uint32_t *ctr, uint32_t key, bool valid) {
  const int lane = (int)__lane_id();
  const uint32_t prev = __shfl_up(key, 1);
  const bool head = valid && (lane == 0 || prev != key);
  const uint64_t heads = __ballot(head);
  const uint64_t valids = __ballot(valid);
  if (heads == 0) return 0;
  const uint64_t le = heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
  const int myhead = le ? 63 - __clzll((long long)le) : 0;
  const uint64_t above = heads & (myhead == 63 ? 0ull : ~((2ull << myhead) - 1ull));
  const int endl = above ? __ffsll((long long)above) - 1 : 64 - __clzll((long long)valids);
  uint32_t base = 0;
  if (head) base = atomicAdd(ctr, (uint32_t)(endl - myhead));
  base = __shfl(base, myhead);
  return base + (uint32_t)(lane - myhead);
}

// counts in key order from the spread counters
__global__ void k_unspread(const uint32_t *spread, uint32_t s, uint32_t nkeys, uint32_t *hist) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nkeys) hist[k] = spread[(k & 15u) * s + (k >> 4)];
}

// One parcel per thread.  The level table and levels are read from global
// memory (cache resident): staging them in LDS per block would cost more
// than the parcel data itself, as each parcel needs one table entry.
__global__ __launch_bounds__(kBlock) void k_sort_keys(const SortArgs a) {
  const int lb = logical_block((int)blockIdx.x, a.per_xcd);
  if (lb >= a.nblk) return;
  const int64_t i = (int64_t)lb * kBlock + threadIdx.x;
  const bool valid = i < a.n;
  uint32_t key = 0xFFFFFFFFu;
  const uint32_t step = a.step + (a.step_dev ? *a.step_dev : 0u);
  if (valid) {
    const double lon = a.lon[i], lat = a.lat[i], p = a.p[i];
    if (!finite3(lon, lat, p)) {
      key = a.nkeys - 1;
    } else if (a.scen && (int64_t)step < (int64_t)a.release[a.scen[i]]) {
      key = a.ntx * a.nty * a.ntz + (uint32_t)a.rank[a.scen[i]];
    } else {
      const double lam = lon - 360.0 * floor((lon - a.lon0) * (1.0 / 360.0));
      int i0 = (int)floor((lam - a.lon0) * a.inv_dlon);
      if (i0 >= a.nx) i0 -= a.nx;
      if (i0 < 0) i0 += a.nx;
      const double phi = fmin(fmax(lat, a.lat0), a.lat_hi);
      int j = (int)floor((phi - a.lat0) * a.inv_dlat);
      j = min(max(j, 0), a.ny - 2);
      const double pc = fmin(fmax(p, a.p_top), a.p_bot);
      int b = (int)((__log2f((float)pc) - a.lut_lo) * a.lut_scale);
      b = min(max(b, 0), kLutBins - 1);
      int k = a.lut[b];
      while (k < a.nz - 2 && a.plev[k + 1] >= pc) ++k;
      while (k > 0 && a.plev[k] < pc) --k;
      key = ((uint32_t)(k >> 2) * a.nty + (uint32_t)(j >> 3)) * a.ntx + (uint32_t)(i0 >> 3);
    }
  }
  // counters of consecutive keys sit spread_s apart: nearly sorted parcels
  // bump consecutive keys, and atomics on one cache line queue up
  const uint32_t rank = wave_run_add(a.spread + (key & 15u) * a.spread_s + (key >> 4), key, valid);
  if (valid) {
    a.keys[i] = key;
    a.ranks[i] = rank;
  }
}

// Exclusive scan, phase 1: each block scans kScanChunk entries in place
// and records the chunk total.
__global__ __launch_bounds__(256) void k_scan_local(uint32_t *data, uint32_t n, uint32_t *sums) {
  __shared__ uint32_t s[256];
  const uint32_t base = blockIdx.x * kScanChunk + threadIdx.x * 4;
  uint32_t v[4];
  uint32_t t = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    v[q] = (base + q < n) ? data[base + q] : 0u;
    t += v[q];
  }
  s[threadIdx.x] = t;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {       // Hillis-Steele inclusive scan
    const uint32_t x = ((int)threadIdx.x >= off) ? s[threadIdx.x - off] : 0u;
    __syncthreads();
    s[threadIdx.x] += x;
    __syncthreads();
  }
  uint32_t run = s[threadIdx.x] - t;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (base + q < n) data[base + q] = run;
    run += v[q];
  }
  if (threadIdx.x == 255) sums[blockIdx.x] = s[255];
}

// Phase 2: one block scans the chunk totals (any count) exclusively.
__global__ __launch_bounds__(256) void k_scan_sums(uint32_t *sums, uint32_t nb) {
  __shared__ uint32_t s[256];
  uint32_t carry = 0;
  for (uint32_t start = 0; start < nb; start += 256) {
    const uint32_t q = start + threadIdx.x;
    const uint32_t v = q < nb ? sums[q] : 0u;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const uint32_t x = ((int)threadIdx.x >= off) ? s[threadIdx.x - off] : 0u;
      __syncthreads();
      s[threadIdx.x] += x;
      __syncthreads();
    }
    if (q < nb) sums[q] = carry + s[threadIdx.x] - v;
    const uint32_t total = s[255];
    __syncthreads();
    carry += total;
  }
}

// Phase 3: add each chunk's prefix.
__global__ __launch_bounds__(256) void k_scan_add(uint32_t *data, uint32_t n, const uint32_t *sums) {
  const uint32_t add = sums[blockIdx.x];
  const uint32_t base = blockIdx.x * kScanChunk + threadIdx.x * 4;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (base + q < n) data[base + q] += add;
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *dst, uint32_t n) {
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) dst[q] = 0u;
}

__global__ __launch_bounds__(kBlock) void k_sort_scatter(const ScatterArgs a) {
  const int lb = logical_block((int)blockIdx.x, a.per_xcd);
  if (lb >= a.nblk) return;
  const int64_t i = (int64_t)lb * kBlock + threadIdx.x;
  if (i >= a.n) return;
  const uint32_t pos = a.offsets[a.keys[i]] + a.ranks[i];
  a.lon2[pos] = a.lon[i];
  a.lat2[pos] = a.lat[i];
  a.p2[pos] = a.p[i];
  a.id2[pos] = a.id[i];
  if (a.scen) a.scen2[pos] = a.scen[i];
  if (a.meso_bytes == 8) {
    static_cast<double *>(a.up2)[pos] = static_cast<const double *>(a.up)[i];
    static_cast<double *>(a.vp2)[pos] = static_cast<const double *>(a.vp)[i];
    static_cast<double *>(a.wp2)[pos] = static_cast<const double *>(a.wp)[i];
  } else if (a.meso_bytes == 4) {
    static_cast<float *>(a.up2)[pos] = static_cast<const float *>(a.up)[i];
    static_cast<float *>(a.vp2)[pos] = static_cast<const float *>(a.vp)[i];
    static_cast<float *>(a.wp2)[pos] = static_cast<const float *>(a.wp)[i];
  }
}

size_t scan_block_sums_len(uint32_t nkeys) { return (nkeys + kScanChunk - 1) / kScanChunk; }

hipError_t launch_fill_u32(uint32_t *dst, uint32_t n, hipStream_t stream) {
  unsigned g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g == 0) g = 1;
  hipLaunchKernelGGL(k_fill_u32, dim3(g), dim3(256), 0, stream, dst, n);
  return hipGetLastError();
}

hipError_t launch_scan_u32(uint32_t *data, uint32_t n, uint32_t *block_sums, hipStream_t stream) {
  const uint32_t nb = (uint32_t)scan_block_sums_len(n);
  hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(256), 0, stream, data, n, block_sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, stream, block_sums, nb);
  hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(256), 0, stream, data, n, block_sums);
  return hipGetLastError();
}

hipError_t launch_sort(const SortArgs &sa, const ScatterArgs &xa, hipStream_t stream) {
  const uint32_t nb = (uint32_t)scan_block_sums_len(sa.nkeys);
  unsigned fill_grid = (16u * sa.spread_s + 255) / 256;
  if (fill_grid > 4096) fill_grid = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid), dim3(256), 0, stream, sa.spread, 16u * sa.spread_s);
  hipLaunchKernelGGL(k_sort_keys, dim3((unsigned)(sa.per_xcd * kXcds)), dim3(kBlock), 0, stream, sa);
  hipLaunchKernelGGL(k_unspread, dim3((sa.nkeys + 255) / 256), dim3(256), 0, stream, sa.spread, sa.spread_s,
                     sa.nkeys, sa.hist);
  hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(256), 0, stream, sa.hist, sa.nkeys, sa.block_sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, stream, sa.block_sums, nb);
  hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(256), 0, stream, sa.hist, sa.nkeys, sa.block_sums);
  hipLaunchKernelGGL(k_sort_scatter, dim3((unsigned)(xa.per_xcd * kXcds)), dim3(kBlock), 0, stream, xa);
  return hipGetLastError();
}

}  // namespace mpt
