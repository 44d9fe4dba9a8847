// k_sort.hip -- counting sort of parcels by grid-box tile: tile key, rank
// inside the tile and histogram in one pass, exclusive scan of the
// histogram, then an atomic-free scatter of the whole parcel state into the
// second buffer set at offset[key] + rank.  Parcels that are already nearly
// sorted share keys along a wave's range, so the histogram counter of a key
// is bumped once per run of equal keys within a wave.
#include "mpt_internal.h"

namespace mpt {

constexpr int kScanChunk = 1024;   // entries per scan block (256 threads x 4)

// counts in key order from the spread counters
__global__ void k_unspread(const uint32_t *spread, uint32_t s, uint32_t nkeys, uint32_t *hist) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nkeys) hist[k] = spread[(k & 15u) * s + (k >> 4)];
}

// Tile key: 8 x 8 x 4 cells (lon x lat x level), lon fastest; parcels not
// yet released at the sort's step go behind the tiles in the release order
// of their scenario; non-finite positions last.  The level table and levels
// are read from global memory (cache resident): staging them in LDS per
// block would cost more than the parcel data itself.
//
// Each wave takes kSortPer * 64 consecutive parcels (group q = parcels
// q*64 .. q*64+63 of the wave's range, one per lane), so a thread has
// kSortPer independent parcels in flight.  Runs of equal keys are found over
// the wave's whole range (a run may cross groups); each run adds its length
// to its key's counter once, every atomic of the wave is issued before any
// result is used, and a parcel's rank is the run's old counter value plus
// its place in the run.  Counters of consecutive keys sit spread_s apart:
// nearly sorted parcels bump consecutive keys, and atomics on one cache line
// queue up.
__global__ __launch_bounds__(kBlock) void k_sort_keys(const SortArgs a) {
  const int lb = logical_block((int)blockIdx.x, a.per_xcd);
  if (lb >= a.nblk) return;
  const int lane = (int)__lane_id();
  const int64_t i_w = (int64_t)lb * (kBlock * kSortPer) + (int64_t)(threadIdx.x >> 6) * (64 * kSortPer);
  const uint32_t step = a.step + (a.step_dev ? *a.step_dev : 0u);
  // The tile key of each parcel, computed in stages over the kSortPer parcels
  // so that their dependent loads (position, level table, levels) are in
  // flight together.  Invalid lanes read parcel n-1 and get key 0xFFFFFFFF.
  int64_t ic[kSortPer];
  double lon[kSortPer], lat[kSortPer], p[kSortPer];
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    const int64_t i = i_w + q * 64 + lane;
    ic[q] = i < a.n ? i : a.n - 1;
    lon[q] = a.lon[ic[q]];
    lat[q] = a.lat[ic[q]];
    p[q] = a.p[ic[q]];
  }
  uint32_t key[kSortPer];
  double pc[kSortPer];
  int k[kSortPer], ci[kSortPer], cj[kSortPer];
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    const double lam = lon[q] - 360.0 * floor((lon[q] - a.lon0) * (1.0 / 360.0));
    int i0 = (int)floor((lam - a.lon0) * a.inv_dlon);
    if (i0 >= a.nx) i0 -= a.nx;
    if (i0 < 0) i0 += a.nx;
    const double phi = fmin(fmax(lat[q], a.lat0), a.lat_hi);
    int j = (int)floor((phi - a.lat0) * a.inv_dlat);
    j = min(max(j, 0), a.ny - 2);
    ci[q] = i0;
    cj[q] = j;
    pc[q] = fmin(fmax(p[q], a.p_top), a.p_bot);
    int b = (int)((__log2f((float)pc[q]) - a.lut_lo) * a.lut_scale);
    b = min(max(b, 0), kLutBins - 1);
    k[q] = a.lut[b];
  }
  uint16_t sc[kSortPer];
  if (a.scen) {
#pragma unroll
    for (int q = 0; q < kSortPer; ++q) sc[q] = a.scen[ic[q]];
  }
  // Level: the largest k <= nz-2 with plev[k] >= pc.  The table's k is a
  // lower bound up to the FP32 rounding of the bin, so the answer is almost
  // always within k-2 .. k+2: the four levels around k decide up to two
  // steps either way, further steps (rare) walk on.
  double pm[kSortPer], p0[kSortPer], p1[kSortPer], p2[kSortPer];
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    pm[q] = a.plev[max(k[q] - 1, 0)];
    p0[q] = a.plev[k[q]];
    p1[q] = a.plev[min(k[q] + 1, a.nz - 1)];
    p2[q] = a.plev[min(k[q] + 2, a.nz - 1)];
  }
  int32_t rel[kSortPer], rk[kSortPer];
  if (a.scen) {
#pragma unroll
    for (int q = 0; q < kSortPer; ++q) {
      rel[q] = a.release[sc[q]];
      rk[q] = a.rank[sc[q]];
    }
  }
  const int top = a.nz - 2;
  uint64_t heads[kSortPer];
  int nvalid = 0;                     // valid parcels form a prefix of the wave's range
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    int kk = k[q];
    if (kk < top && p1[q] >= pc[q]) {
      ++kk;
      if (kk < top && p2[q] >= pc[q]) {
        ++kk;
        while (kk < top && a.plev[kk + 1] >= pc[q]) ++kk;
      }
    } else if (kk > 0 && p0[q] < pc[q]) {
      --kk;
      if (kk > 0 && pm[q] < pc[q]) {
        --kk;
        while (kk > 0 && a.plev[kk] < pc[q]) --kk;
      }
    }
    key[q] = cell_key(ci[q], cj[q], kk, a.ntx, a.nty);
    if (a.scen && (int64_t)step < (int64_t)rel[q]) key[q] = a.ntx * a.nty * a.ntz * kSubKeys + (uint32_t)rk[q];
    if (!finite3(lon[q], lat[q], p[q])) key[q] = a.nkeys - 1;
    const bool valid = i_w + q * 64 + lane < a.n;
    if (!valid) key[q] = 0xFFFFFFFFu;
    uint32_t prev = __shfl_up(key[q], 1);
    if (q > 0) {
      const uint32_t last = __shfl(key[q - 1], 63);   // read with every lane active
      if (lane == 0) prev = last;
    } else if (lane == 0) {
      prev = ~key[q];
    }
    heads[q] = __ballot(valid && prev != key[q]);
    nvalid += __popcll(__ballot(valid));
  }
  // run ends and the atomics, all issued before any result is waited for
  uint32_t base[kSortPer];
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);   // lanes <= lane
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    base[q] = 0;
    if ((heads[q] >> lane) & 1ull) {
      const uint64_t above = heads[q] & ~upto;
      int end = nvalid;
      if (above) {
        end = q * 64 + __ffsll((long long)above) - 1;
      } else {
#pragma unroll
        for (int r = kSortPer - 1; r > q; --r)
          if (heads[r]) end = r * 64 + __ffsll((long long)heads[r]) - 1;
      }
      base[q] = atomicAdd(a.spread + (key[q] & 15u) * a.spread_s + (key[q] >> 4),
                          (uint32_t)(end - (q * 64 + lane)));
    }
  }
  uint32_t cbase = 0;                 // base and wave position of the last head so far
  int cpos = 0;
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    const int64_t i = i_w + q * 64 + lane;
    const uint64_t le = heads[q] & upto;
    const int h = le ? 63 - __clzll((long long)le) : 0;   // the lane's run head in this group
    const uint32_t hb = __shfl(base[q], h);                // read with every lane active
    const uint32_t rank = le ? hb + (uint32_t)(lane - h) : cbase + (uint32_t)(q * 64 + lane - cpos);
    if (heads[q]) {                   // uniform
      const int hl = 63 - __clzll((long long)heads[q]);
      cbase = __shfl(base[q], hl);
      cpos = q * 64 + hl;
    }
    if (i < a.n) {
      a.keys[i] = key[q];
      a.ranks[i] = rank;
    }
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

// One parcel per thread: from i to offset[key] + rank.
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

hipError_t launch_clear_spread(uint32_t *spread, uint32_t spread_s, hipStream_t stream) {
  unsigned fill_grid = (16u * spread_s + 255) / 256;
  if (fill_grid > 4096) fill_grid = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid), dim3(256), 0, stream, spread, 16u * spread_s);
  return hipGetLastError();
}

// The sorted order as a list instead of a move: src[offsets[key] + rank] = i
// (the step launch that follows reads its parcels through it).
__global__ __launch_bounds__(kBlock) void k_sort_inverse(const ScatterArgs a) {
  const int lb = logical_block((int)blockIdx.x, a.per_xcd);
  if (lb >= a.nblk) return;
  const int64_t i = (int64_t)lb * kBlock + threadIdx.x;
  if (i >= a.n) return;
  a.src[a.offsets[a.keys[i]] + a.ranks[i]] = (uint32_t)i;
}

hipError_t launch_sort(const SortArgs &sa, const ScatterArgs &xa, bool keys_done, hipStream_t stream) {
  const uint32_t nb = (uint32_t)scan_block_sums_len(sa.nkeys);
  if (!keys_done) {
    const hipError_t e = launch_clear_spread(sa.spread, sa.spread_s, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sort_keys, dim3((unsigned)(sa.per_xcd * kXcds)), dim3(kBlock), 0, stream, sa);
  }
  hipLaunchKernelGGL(k_unspread, dim3((sa.nkeys + 255) / 256), dim3(256), 0, stream, sa.spread, sa.spread_s,
                     sa.nkeys, sa.hist);
  hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(256), 0, stream, sa.hist, sa.nkeys, sa.block_sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, stream, sa.block_sums, nb);
  hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(256), 0, stream, sa.hist, sa.nkeys, sa.block_sums);
  if (xa.src)
    hipLaunchKernelGGL(k_sort_inverse, dim3((unsigned)(xa.per_xcd * kXcds)), dim3(kBlock), 0, stream, xa);
  else
    hipLaunchKernelGGL(k_sort_scatter, dim3((unsigned)(xa.per_xcd * kXcds)), dim3(kBlock), 0, stream, xa);
  return hipGetLastError();
}

}  // namespace mpt
