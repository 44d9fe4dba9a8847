// k_step.hip -- the fused particle time step (advection, position,
// turbulent and mesoscale diffusion, position) for one or more steps per
// launch, one parcel per thread, state held in registers across steps.
//
// Three launch shapes, each compiled as its own kernel so that each gets its
// own register allocation (sharing one body spills the launch arguments to
// VGPR lanes): one block per 256 parcels (XCD-aware order); a persistent grid
// that walks 256-parcel chunks of the active prefix of a scenario run, whose
// length it reads from device memory; the same walk over a device list of
// parcel indices in increasing order, whose length it reads from device
// memory.  Convection and sedimentation are compiled into kernels of their
// own (k_step_phys_*), so the plain kernels keep their code and registers.
#include "mpt_device.h"
#include "mpt_internal.h"
#include "mpt_stage.h"

namespace mpt {

// The launch arguments re-read from the kernel-argument segment (the step
// kernels take one StepArgs, the segment's first explicit argument, at
// offset 0).  The pointer is opaque to the compiler, so the values loaded
// through it are scalar loads placed where they are used, not values held
// in scalar registers across the whole kernel (there are more of them than
// registers, and the rest would go to VGPR lanes).
__device__ __forceinline__ const StepArgs &reload_args() {
  using CP = const __attribute__((address_space(4))) StepArgs *;
  CP q = (CP)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(q));
  return *(const StepArgs *)q;
}

// Whether a step kernel makes the step's random draws during the
// advection's staging loads (both in the shadow of the one staging per
// step) instead of just before their use.  The draws then stay live across
// the advection: only the FP32 arithmetic forms with FP32 or FP16 fields
// (four waves per SIMD), no convection or sedimentation and one block per
// 256 parcels (launch shape M 0) have the registers for them.
template <int M, int F, typename R, bool P>
struct EarlyDraws {
  static constexpr bool value = M == 0 && (F == kF32 || F == kF16) && sizeof(R) == 4 && !P;
};

// Whether a step kernel stages its winds once per step (advect_block_one):
// the FP64 form and the FP32 arithmetic form with FP32 or FP16 fields,
// launched one block per 256 parcels, without convection or sedimentation.
// Their pairs take the wide box region (Wide: for FP64 the memory of its
// one-time planes, for FP32 and FP16 fields a region wider than those).
// The BF16 form runs five waves per SIMD, whose LDS share leaves no room
// for the pairs, and stages twice.
template <int M, int F, typename R, bool P>
struct OneStaging {
  static constexpr bool value = M == 0 && !P && (sizeof(R) == 8 || F == kF32 || F == kF16);
  static constexpr bool wide = value;
};

// Advances parcel i (valid: the thread holds a parcel; M: the launch shape)
// with the launch's
// arguments (reload_args); lon, lat, p receive
// its final position.  Every thread of the block calls it and runs the same
// steps: the advection's winds are staged for the whole block
// (mpt_stage.h), with barriers inside.
template <int M, int F, typename R, bool P>
__device__ __forceinline__ void step_parcel(const StepLds<R> &sm, const uint16_t *s_lut,
                                            int64_t i, bool valid, uint32_t step0, BoxRef ref, double &lon,
                                            double &lat, double &p) {
  const StepArgs &a = reload_args();
  lon = lat = p = 0.0;
  bool live = false;
  uint32_t id = 0;
  int64_t rel = INT64_MIN;
  const bool do_meso = (a.flags & kMeso) != 0;
  // deferred sort: the whole state moves, so all of it is read
  const bool moving = a.src != nullptr;
  R up = 0, vp = 0, wp = 0;
  if (valid && moving) {                    // every field at once (no scenarios here)
    const int64_t j = (int64_t)a.src[i];
    lon = a.lon[j];
    lat = a.lat[j];
    p = a.p[j];
    id = a.id[j];
    if (a.up) {
      up = static_cast<const R *>(a.up)[j];
      vp = static_cast<const R *>(a.vp)[j];
      wp = static_cast<const R *>(a.wp)[j];
    }
    live = finite3(lon, lat, p);
  } else if (valid) {
    lon = a.lon[i];
    lat = a.lat[i];
    p = a.p[i];
    live = finite3(lon, lat, p);
    if (live) {
      id = a.id[i];
      if (a.scen) rel = a.release[a.scen[i]];
      if (do_meso) {
        up = static_cast<const R *>(a.up)[i];
        vp = static_cast<const R *>(a.vp)[i];
        wp = static_cast<const R *>(a.wp)[i];
      }
    }
  }
  bool moved = false;
  const int nsteps = a.nsteps;
  TimeTable tt;
  for (int s = 0; s < nsteps; ++s) {
    const StepArgs &a = reload_args();
    const uint32_t step = step0 + (uint32_t)s;
    const int e = 2 * (s % kTimeTableSteps);
    if (e == 0) tt = time_table(a, step);            // uniform
    const TimeLoc T0 = time_at(tt, e), T1 = time_at(tt, e + 1);
    const bool act = live && (int64_t)step >= rel && finite3(lon, lat, p);
    moved = moved || act;
    if constexpr (EarlyDraws<M, F, R, P>::value) {
      // the step's random draws depend on (id, step) only: each is made
      // while one of the advection's staging loads is in flight
      R xt[3], xm[3];
      auto draw_turb = [&] { if (a.flags & kTurb) normals3<R>(a.seed, id, step, 0u, xt); };
      auto draw_meso = [&] { if (do_meso) normals3<R>(a.seed, id, step, 1u, xm); };
      static_assert(OneStaging<M, F, R, P>::value, "the early draws ride on the one staging per step");
      if (a.flags & kAdvect) {
        auto draws = [&] {
          draw_turb();
          draw_meso();
        };
        advect_block_one_fill<F, R, OneStaging<M, F, R, P>::wide>(a, sm, s_lut, act, T0, T1, lon, lat, p, ref,
                                                                  draws);
        if (act) position(a, lon, lat, p);
      } else {
        draw_turb();
        draw_meso();
      }
      if (act && (a.flags & (kTurb | kMeso))) {
        if (a.flags & kTurb) turb_drawn<R>(a, xt, lon, lat, p);
        if (do_meso) meso_drawn<F, R>(a, sm.plev, sm.idp, s_lut, xm, T1, lon, lat, p, up, vp, wp);
        position(a, lon, lat, p);
      }
    } else {
      if (a.flags & kAdvect) {
        if constexpr (OneStaging<M, F, R, P>::value) advect_block_one<F, R>(a, sm, s_lut, act, T0, T1, lon, lat, p, ref);
        else advect_block<F, R>(a, sm, s_lut, act, T0, T1, lon, lat, p, ref);
        if (act) position(a, lon, lat, p);
      }
      if (act && (a.flags & (kTurb | kMeso))) {
        if (a.flags & kTurb) turb<R>(a, id, step, lon, lat, p);
        if (do_meso) meso<F, R>(a, sm.plev, sm.idp, s_lut, id, step, T1, lon, lat, p, up, vp, wp);
        position(a, lon, lat, p);
      }
    }
    if constexpr (P) {
      if (act && (a.flags & (kConv | kSedi))) {
        const double t_mid = a.t_start + (double)step * a.dt + 0.5 * a.dt;
        if (a.flags & kConv) convection<F, R>(a, sm.plev, sm.idp, s_lut, id, step, t_mid, lon, lat, p);
        if (a.flags & kSedi) sedimentation<F, R>(a, sm.plev, sm.idp, s_lut, t_mid, lon, lat, p);
        position(a, lon, lat, p);
      }
    }
  }
  const StepArgs &b = reload_args();
  if (b.src) {
    if (!valid) return;
    b.lon_o[i] = lon;
    b.lat_o[i] = lat;
    b.p_o[i] = p;
    b.id_o[i] = id;
    if (b.up) {
      static_cast<R *>(b.up_o)[i] = up;
      static_cast<R *>(b.vp_o)[i] = vp;
      static_cast<R *>(b.wp_o)[i] = wp;
    }
    return;
  }
  if (!moved) return;
  b.lon[i] = lon;
  b.lat[i] = lat;
  b.p[i] = p;
  if (do_meso) {
    static_cast<R *>(b.up)[i] = up;
    static_cast<R *>(b.vp)[i] = vp;
    static_cast<R *>(b.wp)[i] = wp;
  }
}

// Number of parcels a persistent launch must walk: the active prefix left
// by the last sort, extended by the pending scenarios released by `last`.
__device__ __forceinline__ int64_t active_bound(const StepArgs &a, uint32_t last) {
  int lo = 0, hi = a.nscen;              // r = #(rel_sorted[r] <= last)
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)a.rel_sorted[mid] <= (int64_t)last) lo = mid + 1; else hi = mid;
  }
  const int64_t b = a.offsets[a.ntiles + (uint32_t)lo];   // start of the first pending bucket
  return b < a.n ? b : a.n;
}

// Minimum waves per SIMD the compiler must allow (register budget) for the
// FP64 and FP32-arithmetic step kernels: 3 for FP64; in the XCD-block shape
// 5 for BF16 storage (it spills 12 bytes per lane at 96 registers, and the
// extra wave hides more of the staging), 4 for F32 (at 5 it spills 44
// bytes per lane, a loss once the launch also moves the sorted state) and
// FP16 storage (72 bytes); 4 for the persistent and index-list shapes and
// the physics kernels.
#ifndef MPT_WAVES_F64
#define MPT_WAVES_F64 3
#endif
#ifndef MPT_WAVES_F32
#define MPT_WAVES_F32 4
#endif
template <int M, int F>
struct StepWaves {
  static constexpr int value = (M == 0 && F == kBF16) ? 5 : MPT_WAVES_F32;
};

enum : int { kModeBlock = 0, kModePersistent = 1, kModeIndex = 2 };

// The sort key and rank of parcel i's final position, for the sort that
// follows the launch.  Every lane of the wave calls it (valid: lane holds a
// parcel).
__device__ __forceinline__ void leave_sort_key(const StepArgs &a, const double *s_plev,
                                               const uint16_t *s_lut, int64_t i, bool valid, double lon,
                                               double lat, double p) {
  const SortKeyArgs sk = *a.sk;
  const uint32_t key = valid ? tile_key(a, sk, s_plev, s_lut, lon, lat, p) : 0xFFFFFFFFu;
  const uint32_t rank = wave_key_rank(sk, key, valid);
  if (valid) {
    sk.keys[i] = key;
    sk.ranks[i] = rank;
  }
}

template <int M, int F, typename R, bool P>
__device__ __forceinline__ void step_body(const StepArgs &a) {
  __shared__ __attribute__((aligned(16))) uint16_t s_lut[kLutBins];
  const StepLds<R> sm = step_lds<R>(a.nz, F != kF32, OneStaging<M, F, R, P>::wide);
  for (int q = threadIdx.x; q < a.nz; q += kBlock) {
    sm.plev[q] = a.plev[q];
    sm.idp[q] = (q < a.nz - 1) ? a.inv_dp[q] : 0.0;
  }
  static_assert(kLutBins % 8 == 0, "the level table is copied in 16-byte units");
  {                                   // 8 KB in 16-byte units (the table is 256-byte aligned)
    const uint4 *src = reinterpret_cast<const uint4 *>(a.lut);
    uint4 *dst = reinterpret_cast<uint4 *>(s_lut);
    for (int q = threadIdx.x; q < kLutBins / 8; q += kBlock) dst[q] = src[q];
  }
  const uint32_t step0 = a.step0 + (a.step_dev ? *a.step_dev : 0u);
  if constexpr (F != kF32) stage_scale_window(a, met_level(a, a.t_start + (double)step0 * a.dt));
  __syncthreads();
  if constexpr (M == kModeIndex) {
    // a list of parcel indices in increasing order: XCD x owns an even share
    // of its 256-entry chunks (a region of the sorted parcels) and its
    // blocks stride through that share
    const int64_t cnt = *a.index_count;
    const int64_t nchunks = (cnt + kBlock - 1) / kBlock;
    const int xcd = (int)blockIdx.x % kXcds;
    const int q = (int)blockIdx.x / kXcds, nq = (int)gridDim.x / kXcds;
    const int64_t c_lo = nchunks * xcd / kXcds, c_hi = nchunks * (xcd + 1) / kXcds;
    for (int64_t c = c_lo + q; c < c_hi; c += nq) {   // uniform over the block
      const int64_t j = c * kBlock + threadIdx.x;
      double lon, lat, p;
      const bool valid = j < cnt;
      const int64_t i = valid ? (int64_t)a.index[j] : 0;
      const int64_t j0 = c * kBlock;
      const BoxRef ref = block_ref(a, sm.plev, s_lut, j0 < cnt ? (int64_t)a.index[j0] : 0, j0 < cnt);
      step_parcel<M, F, R, P>(sm, s_lut, i, valid, step0, ref, lon, lat, p);
      const StepArgs &b = reload_args();
      if (b.sk) leave_sort_key(b, sm.plev, s_lut, i, valid, lon, lat, p);   // uniform
    }
  } else if constexpr (M == kModeBlock) {
    const int lb = logical_block((int)blockIdx.x, a.per_xcd);
    if (lb >= a.nblk) return;
    const int64_t i = (int64_t)lb * kBlock + threadIdx.x;
    double lon, lat, p;
    const bool valid = i < a.n;
    const BoxRef ref = block_ref(a, sm.plev, s_lut, (int64_t)lb * kBlock, true);
    step_parcel<M, F, R, P>(sm, s_lut, i, valid, step0, ref, lon, lat, p);
    const StepArgs &b = reload_args();
    if (b.sk) leave_sort_key(b, sm.plev, s_lut, i, valid, lon, lat, p);     // uniform
  } else {
    // persistent: XCD x owns an even share of the chunks of the prefix and
    // its blocks stride through that share
    const int64_t bound = active_bound(a, step0 + (uint32_t)(a.nsteps - 1));
    const int64_t nchunks = (bound + kBlock - 1) / kBlock;
    const int xcd = (int)blockIdx.x % kXcds;
    const int q = (int)blockIdx.x / kXcds, nq = (int)gridDim.x / kXcds;
    const int64_t c_lo = nchunks * xcd / kXcds, c_hi = nchunks * (xcd + 1) / kXcds;
    for (int64_t c = c_lo + q; c < c_hi; c += nq) {   // uniform over the block
      const int64_t i = c * kBlock + threadIdx.x;
      double lon, lat, p;
      const BoxRef ref = block_ref(a, sm.plev, s_lut, c * kBlock, true);
      step_parcel<M, F, R, P>(sm, s_lut, i, i < bound, step0, ref, lon, lat, p);
    }
  }
}

template <int M>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(MPT_WAVES_F64)))
void k_step_f64(const StepArgs a) {
  step_body<M, kF32, double, false>(a);
}

template <int M, int F>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(StepWaves<M, F>::value)))
void k_step_f32(const StepArgs a) {
  step_body<M, F, float, false>(a);
}

template <int M>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(MPT_WAVES_F64)))
void k_step_phys_f64(const StepArgs a) {
  step_body<M, kF32, double, true>(a);
}

template <int M, int F>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(MPT_WAVES_F32)))
void k_step_phys_f32(const StepArgs a) {
  step_body<M, F, float, true>(a);
}

// Dynamic LDS of the step kernels (mpt_stage.h).
template <typename R>
static size_t lds_bytes(int field, const StepArgs &a, bool wide = false) {
  return step_lds_bytes<R>(a.nz, field != kF32, wide);
}

template <int M>
static hipError_t launch_mode(int field, int math_f64, const StepArgs &args, dim3 grid,
                              hipStream_t stream) {
  const dim3 block(kBlock);
  if (math_f64) {
    if (field != kF32) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_step_f64<M>, grid, block,
                       lds_bytes<double>(field, args, OneStaging<M, kF32, double, false>::wide), stream, args);
  } else if (field == kF32) {
    hipLaunchKernelGGL((k_step_f32<M, kF32>), grid, block,
                       lds_bytes<float>(field, args, OneStaging<M, kF32, float, false>::wide), stream, args);
  } else if (field == kBF16) {
    hipLaunchKernelGGL((k_step_f32<M, kBF16>), grid, block, lds_bytes<float>(field, args), stream, args);
  } else {
    hipLaunchKernelGGL((k_step_f32<M, kF16>), grid, block,
                       lds_bytes<float>(field, args, OneStaging<M, kF16, float, false>::wide), stream, args);
  }
  return hipGetLastError();
}

// Convection / sedimentation kernels: block and persistent shapes only.
template <int M>
static hipError_t launch_phys(int field, int math_f64, const StepArgs &args, dim3 grid,
                              hipStream_t stream) {
  const dim3 block(kBlock);
  if (math_f64) {
    if (field != kF32) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_step_phys_f64<M>, grid, block, lds_bytes<double>(field, args), stream, args);
  } else if (field == kF32) {
    hipLaunchKernelGGL((k_step_phys_f32<M, kF32>), grid, block, lds_bytes<float>(field, args), stream, args);
  } else if (field == kBF16) {
    hipLaunchKernelGGL((k_step_phys_f32<M, kBF16>), grid, block, lds_bytes<float>(field, args), stream, args);
  } else {
    hipLaunchKernelGGL((k_step_phys_f32<M, kF16>), grid, block, lds_bytes<float>(field, args), stream, args);
  }
  return hipGetLastError();
}

hipError_t launch_step(int field, int math_f64, const StepArgs &args, hipStream_t stream) {
  const dim3 grid((unsigned)(args.persistent ? args.nblk : args.per_xcd * kXcds));
  // R16 storage: the launch's times must fit the scale window
  if (field != kF32 && !r16_launch_fits(args.nsteps, args.dt, args.dt_met)) return hipErrorInvalidValue;
  if (args.flags & (kConv | kSedi)) {
    if (args.index) return hipErrorInvalidValue;
    if (args.persistent) return launch_phys<kModePersistent>(field, math_f64, args, grid, stream);
    return launch_phys<kModeBlock>(field, math_f64, args, grid, stream);
  }
  if (args.index) return launch_mode<kModeIndex>(field, math_f64, args, grid, stream);
  if (args.persistent) return launch_mode<kModePersistent>(field, math_f64, args, grid, stream);
  return launch_mode<kModeBlock>(field, math_f64, args, grid, stream);
}

__global__ void k_add_u32(uint32_t *p, uint32_t v) { *p += v; }
__global__ void k_set_u32(uint32_t *p, uint32_t v) { *p = v; }

hipError_t launch_set_u32(uint32_t *p, uint32_t v, hipStream_t stream) {
  hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, stream, p, v);
  return hipGetLastError();
}

hipError_t launch_add_u32(uint32_t *p, uint32_t v, hipStream_t stream) {
  hipLaunchKernelGGL(k_add_u32, dim3(1), dim3(1), 0, stream, p, v);
  return hipGetLastError();
}

}  // namespace mpt
