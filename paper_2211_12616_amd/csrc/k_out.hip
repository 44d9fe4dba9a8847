// k_out.hip -- gridded output: per box of a regular lon x lat x pressure-
// layer grid, the number of parcels, the sum of their masses and the mass
// mixing ratio (the gridded-data output function of the model's output
// section; the box assignment is stated in include/mpt.h).
//
#include "mpt_device.h"
#include "mpt_internal.h"

namespace mpt {

// Box index of a parcel, or -1 when it is outside the grid or not finite.
__device__ __forceinline__ int32_t out_box(const OutArgs &o, double lon, double lat, double p) {
  if (!finite3(lon, lat, p)) return -1;
  const double x = floor((lon - o.lon0) / o.dlon);
  int64_t i = (int64_t)x % o.nx;
  if (i < 0) i += o.nx;
  const double y = floor((lat - o.lat0) / o.dlat);
  int32_t j;
  if (y < 0.0) return -1;
  if (y >= (double)o.ny) {
    if (lat != o.lat0 + o.ny * o.dlat) return -1;
    j = o.ny - 1;
  } else {
    j = (int32_t)y;
  }
  const double *pe = o.pedges;
  if (!(p <= pe[0] && p > pe[o.nz])) return -1;
  int lo = 0, hi = o.nz - 1;               // largest k with pe[k] >= p
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pe[mid] >= p) lo = mid; else hi = mid - 1;
  }
  return ((int32_t)lo * o.ny + j) * o.nx + (int32_t)i;
}

// A block takes kOutPer * kBlock consecutive parcels and accumulates them
// in an LDS table of kOutSlots boxes (slot claimed by compare-and-swap on
// the box index, a multiplicative hash picks the slot; a parcel whose slot
// holds another box goes straight to memory), then adds each claimed slot
// to memory once.  Sorted parcels of a block fall into few boxes, so memory
// sees few atomics; atomics on neighbouring boxes share cache lines and
// queue up, which made one atomic per run of a wave slow.
constexpr int kOutSlots = 1024, kOutPer = (int)(kOutParcelsPerBlock / kBlock);
constexpr uint32_t kOutEmpty = 0xFFFFFFFFu;

__global__ __launch_bounds__(kBlock) void k_grid_out(const OutArgs o, uint32_t *counts, double *msum) {
  __shared__ uint32_t skey[kOutSlots], scnt[kOutSlots];
  __shared__ double smass[kOutSlots];
  const int lb = logical_block((int)blockIdx.x, o.per_xcd);
  if (lb >= o.nblk) return;                        // uniform over the block
  for (int s = threadIdx.x; s < kOutSlots; s += kBlock) {
    skey[s] = kOutEmpty;
    scnt[s] = 0u;
    smass[s] = 0.0;
  }
  __syncthreads();
  const int64_t q0 = (int64_t)lb * (kOutPer * kBlock) + threadIdx.x;
#pragma unroll
  for (int r = 0; r < kOutPer; ++r) {
    const int64_t q = q0 + r * kBlock;
    if (q >= o.n) break;
    const int32_t b = out_box(o, o.lon[q], o.lat[q], o.p[q]);
    if (b < 0) continue;
    const double m = o.mass ? o.mass[q] : 1.0;
    const uint32_t slot = ((uint32_t)b * 2654435761u) >> (32 - 10);
    const uint32_t old = atomicCAS(&skey[slot], kOutEmpty, (uint32_t)b);
    if (old == kOutEmpty || old == (uint32_t)b) {
      atomicAdd(&scnt[slot], 1u);
      atomicAdd(&smass[slot], m);
    } else {
      atomicAdd(&counts[b], 1u);
      unsafeAtomicAdd(&msum[b], m);
    }
  }
  __syncthreads();
  for (int s = threadIdx.x; s < kOutSlots; s += kBlock) {
    const uint32_t b = skey[s];
    if (b != kOutEmpty) {
      atomicAdd(&counts[b], scnt[s]);
      unsafeAtomicAdd(&msum[b], smass[s]);
    }
  }
}

// mmr[b] = msum[b] / air mass of box b.
__global__ __launch_bounds__(256) void k_grid_mmr(const OutArgs o, const double *msum, double *mmr) {
  const int64_t nbox = (int64_t)o.nx * o.ny * o.nz;
  const double dl = o.dlon * (kPi / 180.0);
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nbox;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(b / ((int64_t)o.nx * o.ny));
    const int j = (int)((b / o.nx) % o.ny);
    const double s0 = sin((o.lat0 + j * o.dlat) * (kPi / 180.0));
    const double s1 = sin((o.lat0 + (j + 1) * o.dlat) * (kPi / 180.0));
    const double air = kREarth * kREarth * dl * (s1 - s0) * (o.pedges[k] - o.pedges[k + 1]) * 100.0 / kG;
    mmr[b] = msum[b] / air;
  }
}

hipError_t launch_grid_out(const OutArgs &o, uint32_t *counts, double *msum, double *mmr, hipStream_t s) {
  const int64_t nbox = (int64_t)o.nx * o.ny * o.nz;
  // counts, then the FP64 sums as 32-bit words (zero bits are 0.0)
  hipError_t e = launch_fill_u32(counts, (uint32_t)nbox, s);
  if (e != hipSuccess) return e;
  e = launch_fill_u32(reinterpret_cast<uint32_t *>(msum), (uint32_t)(2 * nbox), s);
  if (e != hipSuccess) return e;
  if (o.n > 0)
    hipLaunchKernelGGL(k_grid_out, dim3((unsigned)(o.per_xcd * kXcds)), dim3(kBlock), 0, s, o, counts, msum);
  if (mmr) {
    unsigned nb = (unsigned)((nbox + 255) / 256);
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_grid_mmr, dim3(nb), dim3(256), 0, s, o, msum, mmr);
  }
  return hipGetLastError();
}

}  // namespace mpt
