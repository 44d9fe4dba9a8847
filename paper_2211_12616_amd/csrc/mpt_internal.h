// mpt_internal.h -- launchers shared by the runtime and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpt_device.h"

namespace mpt {

// Step kernels (k_step.hip).  field: FieldKind; math_f64: 1 = FP64 arithmetic.
hipError_t launch_step(int field, int math_f64, const StepArgs &args, hipStream_t stream);

// Met storage (k_met.hip).
hipError_t launch_pack_f32(const float *u, const float *v, const float *w, float4 *dst,
                           int64_t npts, hipStream_t stream);
hipError_t launch_level_absmax(const float *u, const float *v, const float *w, int64_t nxy, int nz,
                               float *scales, hipStream_t stream);
hipError_t launch_pack_r16(int field, const float *u, const float *v, const float *w,
                           const float *scales, ushort4 *dst, int64_t nxy, int nz,
                           hipStream_t stream);
hipError_t launch_fill_f32(float *dst, float value, int64_t n, hipStream_t stream);

// Sort (k_sort.hip).
struct SortArgs {
  const double *lon, *lat, *p;
  const double *plev, *inv_dp;
  int nx, ny, nz;
  double lon0, inv_dlon, lat0, inv_dlat, lat_hi, p_top, p_bot;
  uint32_t ntx, nty, ntz, nkeys;   // nkeys = ntiles + max scenarios + 1
  int64_t n;
  // scenario runs: parcels not yet released at the sort's step go behind the
  // tiles, ordered by the release rank of their scenario; non-finite last
  const uint16_t *scen;            // null: no scenarios
  const int32_t *release, *rank;   // per scenario (device)
  uint32_t step;                   // step the sort precedes (+ *step_dev if set)
  const uint32_t *step_dev;
  uint32_t *keys;
  uint32_t *hist;                  // nkeys counters, then scanned in place
  uint32_t *block_sums;
  int nblk, per_xcd;
};

struct ScatterArgs {
  int64_t n;
  const uint32_t *keys;
  uint32_t *cursor;
  const double *lon, *lat, *p;
  const uint32_t *id;
  const void *up, *vp, *wp;
  const uint16_t *scen;
  double *lon2, *lat2, *p2;
  uint32_t *id2;
  void *up2, *vp2, *wp2;
  uint16_t *scen2;
  int meso_bytes;                  // 8 (double), 4 (float) or 0 (no meso state)
  int nblk, per_xcd;
};

hipError_t launch_sort(const SortArgs &sa, const ScatterArgs &xa, hipStream_t stream);

// Single-word device helpers (k_step.hip).
hipError_t launch_set_u32(uint32_t *p, uint32_t v, hipStream_t stream);
hipError_t launch_add_u32(uint32_t *p, uint32_t v, hipStream_t stream);
size_t scan_block_sums_len(uint32_t nkeys);

}  // namespace mpt
