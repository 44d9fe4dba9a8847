// mpt_internal.h -- launchers shared by the runtime and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpt_device.h"
#include "mpt_window.h"

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
// Temperature into the fourth value of the records of a stored level
// (R16: with the per-level scales t_scales[nz] it computes); surface records.
hipError_t launch_pack_temp(int field, const float *T, float *t_scales, void *dst, int64_t nxy, int nz,
                            hipStream_t stream);
hipError_t launch_pack_sfc(const float *cape, const float *pel, const float *ps, float4 *dst, int64_t nxy,
                           hipStream_t stream);
hipError_t launch_fill_f32(float *dst, float value, int64_t n, hipStream_t stream);
// Spread table of the level pair in ring slots s0 (earlier) and s1 into out
// (level_elems records of {su, sv, sw, 0}: double when f64, else float).
hipError_t launch_cell_sigma(int field, bool f64, const void *met, const float *scales, int s0, int s1,
                             int64_t level_elems, int nx, int ny, int nz, void *out, hipStream_t stream);

// Sort (k_sort.hip).
// Parcels per thread in the sort's key kernel (a block covers
// kSortPer * kBlock parcels).
constexpr int kSortPer = 4;
// The sort's ranks, offsets and scatter positions are 32-bit.
constexpr int64_t kMaxParcels = 0xFFFFFFFFll;

struct SortArgs {
  const double *lon, *lat, *p;
  const double *plev, *inv_dp;
  const uint16_t *lut;
  float lut_lo, lut_scale;
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
  uint32_t *ranks;                 // rank of the parcel among its key's parcels
  uint32_t *hist;                  // nkeys counts in key order, then scanned in place
  uint32_t *spread;                // the counters while keys are counted: key k at
                                   // (k % 16) * spread_s + k / 16
  uint32_t spread_s;               // ceil(nkeys / 16)
  uint32_t *block_sums;
  int nblk, per_xcd;
};

struct ScatterArgs {
  int64_t n;
  const uint32_t *keys;
  const uint32_t *ranks;
  const uint32_t *offsets;         // exclusive scan of the histogram
  const double *lon, *lat, *p;
  const uint32_t *id;
  const void *up, *vp, *wp;
  const uint16_t *scen;
  double *lon2, *lat2, *p2;
  uint32_t *id2;
  void *up2, *vp2, *wp2;
  uint16_t *scen2;
  int meso_bytes;                  // 8 (double), 4 (float) or 0 (no meso state)
  uint32_t *src;                   // not null: write the sorted order here (src[position] =
                                   // parcel index) instead of moving the state
  int nblk, per_xcd;
};

// keys_done: keys, ranks and the spread counters already hold the keys of
// the parcels (a step launch computed them); otherwise the key pass runs.
hipError_t launch_sort(const SortArgs &sa, const ScatterArgs &xa, bool keys_done, hipStream_t stream);
// Zero the spread counters before a launch that counts keys into them.
hipError_t launch_clear_spread(uint32_t *spread, uint32_t spread_s, hipStream_t stream);

// Learned k-step advection surrogate (k_surr.hip).
constexpr int kSurrK = 8;                       // steps per surrogate block
constexpr int kSurrIn = 81, kSurrInPad = 96;    // 3 variables x 27 stencil points
constexpr int kSurrHid = 128;
constexpr int kSurrOut = 3, kSurrOutPad = 16;   // east km, north km, dp hPa
constexpr int kXLd = 104, kHLd = 136;           // LDS row strides (bf16)
// flat FP32 parameters: W[in][out] then bias, per layer
constexpr int kOffW1 = 0, kOffB1 = 12288, kOffW2 = 12416, kOffB2 = 28800, kOffW3 = 28928,
              kOffB3 = 45312, kOffW4 = 45440, kOffB4 = 47488, kSurrNParam = 47504;
constexpr int kWtSize = 47104;                  // bf16 [out][in] copies of W1..W4
constexpr int kWbSize = 34816;                  // bf16 [in][out] copies of W2..W4
// inference LDS image: W1..W4 as [out][in] rows padded by 8, K permuted to
// the order the MLP kernel feeds them
constexpr int kW1Ld = kSurrInPad + 8, kWLd = kSurrHid + 8;
constexpr int kWiSize = kSurrHid * kW1Ld + 2 * kSurrHid * kWLd + kSurrOutPad * kWLd;
constexpr int kSurrMaxBatch = 8192;
constexpr int kSurrStatBlocks = 1024;
constexpr int64_t kSurrChunk = 1 << 22;          // parcels per stencil / MLP / apply pass


struct SurrW {
  const uint16_t *wt1, *wt2, *wt3, *wt4;        // forward fragments, [out][in]
  const uint16_t *wb2, *wb3, *wb4;              // backward fragments, [in][out]
  const float *b1, *b2, *b3, *b4;
  const float *norm;                            // in mean[3], in std[3], out mean[3], out std[3]
  const uint16_t *wi;                           // inference LDS image (loaded weights only)
};

struct SurrTrain {
  const float *x, *y;                           // batch inputs (raw) and targets
  int64_t batch;                                // multiple of 64
  uint16_t *xn, *h1, *h2, *h3, *dy, *dh1, *dh2, *dh3;
  float *yp, *grad, *loss;
};

hipError_t launch_surr_datagen(const StepArgs &a, int64_t n, const double *lon, const double *lat,
                               const double *p, const uint32_t *step, float *x, float *y,
                               hipStream_t s);
hipError_t launch_surr_stats(const float *x, const float *y, int64_t n, double *part, int nblk,
                             float *norm, hipStream_t s);
hipError_t launch_surr_init(float *params, uint64_t seed, hipStream_t s);
hipError_t launch_surr_pack(const float *params, uint16_t *wt, uint16_t *wb, hipStream_t s);
hipError_t launch_surr_pack_inf(const uint16_t *wt, uint16_t *wi, hipStream_t s);
// Stencil rows X (normalized bf16, 96 per row) are stored chunk-major: the
// 16-byte chunk c of row r at X + (c * ldc + r) * 8, ldc >= the rows held.
// raw inputs -> outputs, in chunks of at most `chunk` rows through X
// (bf16 [12][chunk][8])
hipError_t launch_surr_forward(const SurrW &W, const float *x, int64_t n, uint16_t *X, float *y,
                               int64_t chunk, hipStream_t s);
// rows X (n rows, ldc per chunk) -> Y[row * ldy + 0..2]
hipError_t launch_surr_mlp(const SurrW &W, const uint16_t *X, int64_t n, int64_t ldc, float *Y, int ldy,
                           hipStream_t s);
// FP32 field interpolated to time t ([level_elems] float4)
hipError_t launch_surr_tfield(const StepArgs &a, double t, float4 *F, hipStream_t s);
// stencil rows of parcels i0 .. i0 + cnt - 1 (cnt <= ldc) at step a.step0
// from the field F at that step's time
hipError_t launch_surr_x(const StepArgs &a, const SurrW &W, const float4 *F, int64_t i0, int64_t cnt,
                         uint16_t *X, int64_t ldc, hipStream_t s);
// consistency estimate and acceptance for parcels i0 .. i0 + cnt - 1 (i0 a
// multiple of 64); fb_mask[i / 64] gets the wave's ballot of parcels that
// fall back
hipError_t launch_surr_apply(const StepArgs &a, float tau_km, const float *Y, int64_t i0, int64_t cnt,
                             float *err_out, uint64_t *fb_mask, hipStream_t s);
// ordered fallback list: list[0 .. off[nw]) = indices of the set bits of
// fb_mask[0 .. nw), nw = ceil(n / 64), in increasing order; off holds nw + 1
// entries and sums scan_block_sums_len(nw + 1)
hipError_t launch_surr_fblist(const uint64_t *fb_mask, int64_t n, uint32_t *off, uint32_t *sums,
                              uint32_t *list, uint32_t *fallbacks, hipStream_t s);
hipError_t launch_surr_train(const SurrW &W, const SurrTrain &T, float *params, float *m, float *v,
                             float lr, float bc1, float bc2, hipStream_t s);
hipError_t launch_surr_grad(const SurrW &W, const SurrTrain &T, hipStream_t s);

// Gridded output (k_out.hip).
struct OutArgs {
  const double *lon, *lat, *p;
  const double *mass;              // null: unit masses
  int64_t n;
  int nx, ny, nz;
  double lon0, dlon, lat0, dlat;
  const double *pedges;            // device [nz + 1], strictly decreasing
  int nblk, per_xcd;
};
constexpr int64_t kOutParcelsPerBlock = 1024;    // parcels per block of the output kernel
// zero counts and sums, accumulate the parcels, then mmr (if not null)
hipError_t launch_grid_out(const OutArgs &o, uint32_t *counts, double *msum, double *mmr, hipStream_t s);
// dst[0 .. n) = 0 (k_sort.hip)
hipError_t launch_fill_u32(uint32_t *dst, uint32_t n, hipStream_t s);

// Hybrid model levels to pressure levels (k_ml2pl.hip).
struct Ml2PlArgs {
  int nx, ny, nz, nml;             // target grid, number of model levels
  const double *plev;              // device [nz] target pressures
  const double *a, *b;             // device [nml]: p_k = a_k + b_k ps, decreasing with k
};
hipError_t launch_ml_to_pl(const Ml2PlArgs &g, const float *ps, const float *u, const float *v,
                           const float *w, float *uo, float *vo, float *wo, hipStream_t s);

// Single-word device helpers (k_step.hip).
hipError_t launch_set_u32(uint32_t *p, uint32_t v, hipStream_t stream);
hipError_t launch_add_u32(uint32_t *p, uint32_t v, hipStream_t stream);
size_t scan_block_sums_len(uint32_t nkeys);
// exclusive prefix sum of data[0 .. n) in place; block_sums holds
// scan_block_sums_len(n) entries (k_sort.hip)
hipError_t launch_scan_u32(uint32_t *data, uint32_t n, uint32_t *block_sums, hipStream_t stream);

}  // namespace mpt
