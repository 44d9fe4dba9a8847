// mpt_stage.h -- LDS-staged winds for the step kernels.
//
// Parcels are sorted by tiles of 8 x 8 x 4 cells (lon fastest), so the 256
// parcels of a block sit in one tile or in two tiles next to each other in
// longitude.  For each of the two wind evaluations of a midpoint step the
// whole block
//   1. finds the bounding box of the cells its active parcels occupy (wave
//      reductions, then over the four waves through LDS);
//   2. if the box's grid points fit the LDS capacity: loads them from the
//      two time levels with coalesced loads along longitude, weights them in
//      time once per point (the evaluation time is the block's), and stores
//      u, v, w as three planes in LDS;
//   3. lets each parcel read its 8 corners from LDS and interpolate in
//      space.
// A box that does not fit (parcels not sorted, a block spanning the end of a
// tile row, a sparse set) makes the whole block gather its 16 records per
// parcel from global memory instead: the decision is uniform over the block,
// so no wave runs both paths.  Both paths weight each corner in time first
// and then interpolate along lon, lat and p with the same operations, so they
// give the same bits.
//
// Every thread of the block must take part in each evaluation (two barriers
// each), also threads without an active parcel.
//
// block_ref gives the reference cell the first box is measured from.
#pragma once

#include <type_traits>

#include "mpt_device.h"

namespace mpt {

// Capacity of the staged box in grid points: 3 x 4 B (FP32 values) or
// 3 x 8 B (FP64) per point.
template <typename R> struct BoxCap;
template <> struct BoxCap<float> { static constexpr int value = 1280; };
template <> struct BoxCap<double> { static constexpr int value = 1536; };

__host__ __device__ constexpr size_t round16(size_t x) { return (x + 15) & ~(size_t)15; }

// Reduction slots of the box exchange: 8 ints per wave for the exact
// bounds, then 2 per wave for the offset masks.
constexpr int kRedInts = (kBlock / 64) * 8 + (kBlock / 64) * 2 + 8;

// The one staging per step keeps an FP32 pair per point and variable (8
// bytes).  Points of its box: FP64 form 1536 (the memory of its one-time
// planes), FP32 form 1200 (28.8 KB) and FP16-storage form 1000 (24 KB,
// beside its scale window; both four blocks per CU).
constexpr int kWidePairs = 1200;
constexpr int kWidePairsR16 = 1000;
using Pair = float2;
template <typename R>
__host__ __device__ constexpr int wide_pairs(bool r16) {
  return sizeof(R) == 8 ? BoxCap<double>::value : (r16 ? kWidePairsR16 : kWidePairs);
}

// Bytes of the box region: u, v, w planes of BoxCap values each, or (wide)
// also enough for wide_pairs pairs per variable.
template <typename R>
__host__ __device__ constexpr size_t box_bytes(bool wide, bool r16) {
  return round16(wide && (size_t)3 * wide_pairs<R>(r16) * sizeof(Pair) > (size_t)3 * BoxCap<R>::value * sizeof(R)
                     ? (size_t)3 * wide_pairs<R>(r16) * sizeof(Pair)
                     : (size_t)3 * BoxCap<R>::value * sizeof(R));
}

// Dynamic LDS of the step kernels, in this order: the R16 scale window
// (kScaleWin x 3 x nz floats; it starts the dynamic region), the level
// pressures and inverse spacings (nz doubles each), the box region
// (box_bytes) and the reduction slots.
template <typename R>
__host__ __device__ constexpr size_t step_lds_bytes(int nz, bool r16, bool wide = false) {
  return (r16 ? round16((size_t)kScaleWin * 3 * nz * sizeof(float)) : 0) + round16((size_t)2 * nz * sizeof(double)) +
         box_bytes<R>(wide, r16) + (size_t)kRedInts * sizeof(int);
}

template <typename R>
struct StepLds {
  double *plev, *idp;
  R *bu, *bv, *bw;
  int *red;
};

template <typename R>
__device__ __forceinline__ StepLds<R> step_lds(int nz, bool r16, bool wide = false) {
  unsigned char *base = reinterpret_cast<unsigned char *>(s_scale_win);
  size_t off = r16 ? round16((size_t)kScaleWin * 3 * nz * sizeof(float)) : 0;
  StepLds<R> sm;
  sm.plev = reinterpret_cast<double *>(base + off);
  sm.idp = sm.plev + nz;
  off += round16((size_t)2 * nz * sizeof(double));
  sm.bu = reinterpret_cast<R *>(base + off);
  sm.bv = sm.bu + BoxCap<R>::value;
  sm.bw = sm.bv + BoxCap<R>::value;
  off += box_bytes<R>(wide, r16);
  sm.red = reinterpret_cast<int *>(base + off);
  return sm;
}

// The staged box (uniform over the block): grid columns gi .. gi + bi - 1
// (mod nx), rows j0 .. j0 + bj - 1, levels k0 .. k0 + bk - 1.
struct Box {
  int gi, j0, k0, bi, bj, bk;
  bool ok;
};

// Division by a box extent b (2 <= b <= kMaxExtent) of indices q < 2^11:
// q / b == umulhi(q, ceil(2^32 / b)) (the error q (m - 2^32/b) / 2^32 < 2^-21
// stays below 1/b, the distance of a non-integer quotient from the next
// integer).  The magic numbers come from a constant table (scalar loads).
constexpr int kMaxExtent = 256;
struct DivMagic {
  uint32_t m[kMaxExtent + 1];
  constexpr DivMagic() : m() {
    for (int b = 2; b <= kMaxExtent; ++b) m[b] = (uint32_t)((0x100000000ull + (uint64_t)b - 1) / (uint64_t)b);
  }
};
__constant__ constexpr DivMagic kDivMagic{};

// Reference cell of the block's boxes (uniform): the start of the previous
// box, or at a launch's start the origin of the first parcel's tile.
struct BoxRef {
  int i, j, k;
};

// Exact bounding box of the cells of the active lanes of the block.
// Columns are measured from ref.i, the short way round the circle.  Each
// wave reduces its active lanes' offsets (min of the values and of their
// negatives, in each direction); the four waves' results meet in LDS, every
// lane combines them and the box goes to scalar registers.  ref becomes
// the new box's start.  Contains a barrier.
template <typename R>
__device__ __forceinline__ Box block_box_exact(const StepArgs &a, const StepLds<R> &sm, bool act, const Loc<R> &L,
                                               BoxRef &ref) {
  int iref = ref.i;
  constexpr int big = 0x7fffffff;
  const int h = a.nx >> 1;
  int di = L.i0 - iref;
  if (di > h) di -= a.nx;
  else if (di < -h) di += a.nx;
  const int v0 = __ockl_wfred_min_i32(act ? di : big), v1 = __ockl_wfred_min_i32(act ? -di : big);
  const int v2 = __ockl_wfred_min_i32(act ? L.j : big), v3 = __ockl_wfred_min_i32(act ? -L.j : big);
  const int v4 = __ockl_wfred_min_i32(act ? L.k : big), v5 = __ockl_wfred_min_i32(act ? -L.k : big);
  const int w = (int)threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    int4 *r = reinterpret_cast<int4 *>(sm.red) + 2 * w;
    r[0] = make_int4(v0, v1, v2, v3);
    r[1] = make_int4(v4, v5, 0, 0);
  }
  __syncthreads();
  int m[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) m[q] = big;
#pragma unroll
  for (int ww = 0; ww < kBlock / 64; ++ww) {
    const int4 *r = reinterpret_cast<const int4 *>(sm.red) + 2 * ww;
    const int4 x = r[0], y = r[1];
    m[0] = min(m[0], x.x); m[1] = min(m[1], x.y); m[2] = min(m[2], x.z); m[3] = min(m[3], x.w);
    m[4] = min(m[4], y.x); m[5] = min(m[5], y.y);
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) m[q] = __builtin_amdgcn_readfirstlane(m[q]);
  Box b;
  b.ok = false;
  b.gi = b.j0 = b.k0 = 0;
  b.bi = b.bj = b.bk = 2;
  if (m[0] == big) return b;                          // no active parcel
  int gi = iref + m[0];
  if (gi < 0) gi += a.nx;
  else if (gi >= a.nx) gi -= a.nx;
  b.gi = gi;
  b.bi = -m[1] - m[0] + 2;                            // corners i0 and i0 + 1
  b.j0 = m[2];
  b.bj = -m[3] - m[2] + 2;
  b.k0 = m[4];
  b.bk = -m[5] - m[4] + 2;
  b.ok = b.bi <= a.nx && b.bi <= kMaxExtent && b.bj <= kMaxExtent && b.bi * b.bj * b.bk <= BoxCap<R>::value;
  ref.i = b.gi;
  ref.j = b.j0;
  ref.k = b.k0;
  return b;
}

// Bounding box of the cells of the active lanes of the block, from one-hot
// masks of each lane's offsets from the reference cell (columns -3 .. 27,
// rows and levels -3 .. 11; bit 0 marks an offset outside), ORed over the
// wave and over the four waves through LDS: two reductions instead of six.
// A block with an offset outside those ranges (the first box after a sort
// for a block that spans a tile-row end, parcels far apart) takes the exact
// bounds instead.  ref becomes the new box's start.  Contains the block's
// first barrier of the evaluation (two when the exact bounds are needed).
template <typename R>
__device__ __forceinline__ Box block_box(const StepArgs &a, const StepLds<R> &sm, bool act, const Loc<R> &L,
                                         BoxRef &ref) {
  const int h = a.nx >> 1;
  int di = L.i0 - ref.i;
  if (di > h) di -= a.nx;
  else if (di < -h) di += a.nx;
  const int dj = L.j - ref.j, dk = L.k - ref.k;
  uint32_t mi = 0, mjk = 0;
  if (act) {
    mi = (uint32_t)(di + 3) < 31u ? 2u << (di + 3) : 1u;
    const uint32_t mj = (uint32_t)(dj + 3) < 15u ? 2u << (dj + 3) : 1u;
    const uint32_t mk = (uint32_t)(dk + 3) < 15u ? 2u << (dk + 3) : 1u;
    mjk = mj | (mk << 16);
  }
  mi = __ockl_wfred_or_u32(mi);
  mjk = __ockl_wfred_or_u32(mjk);
  int *slots = sm.red + (kBlock / 64) * 8;
  const int w = (int)threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) reinterpret_cast<int2 *>(slots)[w] = make_int2((int)mi, (int)mjk);
  __syncthreads();
  const int4 x = reinterpret_cast<const int4 *>(slots)[0], y = reinterpret_cast<const int4 *>(slots)[1];
  const uint32_t MI = __builtin_amdgcn_readfirstlane((uint32_t)(x.x | x.z | y.x | y.z));
  const uint32_t MJK = __builtin_amdgcn_readfirstlane((uint32_t)(x.y | x.w | y.y | y.w));
  Box b;
  b.ok = false;
  b.gi = b.j0 = b.k0 = 0;
  b.bi = b.bj = b.bk = 2;
  if (MI == 0) return b;                              // no active parcel
  const uint32_t MJ = MJK & 0xFFFFu, MK = MJK >> 16;
  if (((MI | MJ | MK) & 1u) || a.nx > 0xFFFF || a.ny > 0xFFFF) return block_box_exact<R>(a, sm, act, L, ref);
  const int lo_i = __builtin_ctz(MI) - 4, hi_i = 27 - __builtin_clz(MI);
  const int lo_j = __builtin_ctz(MJ) - 4, hi_j = 27 - __builtin_clz(MJ);
  const int lo_k = __builtin_ctz(MK) - 4, hi_k = 27 - __builtin_clz(MK);
  int gi = ref.i + lo_i;
  if (gi < 0) gi += a.nx;
  else if (gi >= a.nx) gi -= a.nx;
  b.gi = gi;
  b.bi = hi_i - lo_i + 2;                             // corners i0 and i0 + 1
  b.j0 = ref.j + lo_j;
  b.bj = hi_j - lo_j + 2;
  b.k0 = ref.k + lo_k;
  b.bk = hi_k - lo_k + 2;
  b.ok = b.bi <= a.nx && b.bi * b.bj * b.bk <= BoxCap<R>::value;
  ref.i = b.gi;
  ref.j = b.j0;
  ref.k = b.k0;
  return b;
}

// The reference cell of a block's first box, the same in every thread: the
// origin of the tile (8 x 8 x 4 cells) holding the block's first parcel
// (index i_first), or cell (0, 0, 0) when there is none or it is not
// finite (any reference is correct; a far one sends the first box to the
// exact bounds).  plev, lut: the level table and its lookup (LDS or global).
__device__ __forceinline__ BoxRef block_ref(const StepArgs &a, const double *plev, const uint16_t *lut,
                                            int64_t i_first, bool valid) {
  BoxRef r{0, 0, 0};
  if (!valid) return r;
  const double lon = a.lon[i_first], lat = a.lat[i_first], p = a.p[i_first];
  if (!finite3(lon, lat, p)) return r;
  const double lam = lon - 360.0 * floor((lon - a.lon0) * (1.0 / 360.0));
  int i0 = (int)floor((lam - a.lon0) * a.inv_dlon);
  if (i0 >= a.nx) i0 -= a.nx;
  if (i0 < 0) i0 += a.nx;
  const double phi = fmin(fmax(lat, a.lat0), a.lat_hi);
  int j = (int)floor((phi - a.lat0) * a.inv_dlat);
  j = min(max(j, 0), a.ny - 2);
  const int k = level_index(a, plev, lut, fmin(fmax(p, a.p_top), a.p_bot));
  r.i = __builtin_amdgcn_readfirstlane(i0 & ~7);
  r.j = __builtin_amdgcn_readfirstlane(j & ~7);
  r.k = __builtin_amdgcn_readfirstlane(k & ~3);
  return r;
}

// Loads the box's points from the two time levels of L (slots l, l1; R16:
// decoded with the scales of levels la and la + 1 from the window), weights
// them in time with L.ft and stores u, v, w in LDS.  Point q of the box is
// column q % bi, row (q / bi) % bj, level q / (bi bj); consecutive threads
// take consecutive columns, so each row is one coalesced run.
template <int F, typename R>
__device__ __forceinline__ void stage_box(const StepArgs &a, const StepLds<R> &sm, const Box &b, const Loc<R> &L) {
  using T = typename Rec<F>::T;
  const T *lev0 = reinterpret_cast<const T *>(a.met) + (size_t)L.l * (size_t)a.level_elems;
  const T *lev1 = reinterpret_cast<const T *>(a.met) + (size_t)L.l1 * (size_t)a.level_elems;
  const int npts = b.bi * b.bj * b.bk;
  const uint32_t mi = kDivMagic.m[b.bi];
  const uint32_t mj = kDivMagic.m[b.bj];
  const float *sw0 = s_scale_win + (L.la % kScaleWin) * 3 * a.nz;
  const float *sw1 = s_scale_win + ((L.la + 1) % kScaleWin) * 3 * a.nz;
  // two points per thread and pass, so that four loads are in flight
  for (int q0 = (int)threadIdx.x; q0 < npts; q0 += 2 * kBlock) {
    T r0[2], r1[2];
    int kq[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q = min(q0 + u * kBlock, npts - 1);   // a duplicate of the last point is harmless
      const int r = (int)__umulhi((uint32_t)q, mi);
      const int ii = q - r * b.bi;
      const int kk = (int)__umulhi((uint32_t)r, mj);
      const int jj = r - kk * b.bj;
      int gi = b.gi + ii;
      if (gi >= a.nx) gi -= a.nx;
      kq[u] = b.k0 + kk;
      const int off = (kq[u] * a.ny + b.j0 + jj) * a.nx + gi;   // < 2^31: nx*ny*nz is
      r0[u] = lev0[off];
      r1[u] = lev1[off];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      // the clamped duplicate of the last point stores that point's own
      // value again: no branch, so the compiler keeps both points' loads
      // ahead of the first use instead of sinking the second into a branch
      const int q = min(q0 + u * kBlock, npts - 1);
      const int k = kq[u];
      float sc0[3] = {1.0f, 1.0f, 1.0f}, sc1[3] = {1.0f, 1.0f, 1.0f};
      if constexpr (F != kF32) {
        sc0[0] = sw0[k]; sc0[1] = sw0[a.nz + k]; sc0[2] = sw0[2 * a.nz + k];
        sc1[0] = sw1[k]; sc1[1] = sw1[a.nz + k]; sc1[2] = sw1[2 * a.nz + k];
      }
      R v0[3], v1[3];
      Fetch<F, R>::get(r0[u], sc0, v0);
      Fetch<F, R>::get(r1[u], sc1, v1);
      sm.bu[q] = lerp(v0[0], v1[0], L.ft);
      sm.bv[q] = lerp(v0[1], v1[1], L.ft);
      sm.bw[q] = lerp(v0[2], v1[2], L.ft);
    }
  }
}

// The 8 time-weighted corners of L's cell from the staged box, then the
// spatial interpolation.
template <typename R>
__device__ __forceinline__ void interp_box(const StepArgs &a, const StepLds<R> &sm, const Box &b, const Loc<R> &L,
                                           R out[3]) {
  int ci = L.i0 - b.gi;
  if (ci < 0) ci += a.nx;
  const int sj = b.bi, sk = b.bi * b.bj;
  const int base = (L.k - b.k0) * sk + (L.j - b.j0) * sj + ci;
  R cv[2][2][2][3];
#pragma unroll
  for (int dk = 0; dk < 2; ++dk)
#pragma unroll
    for (int dj = 0; dj < 2; ++dj)
#pragma unroll
      for (int di = 0; di < 2; ++di) {
        const int q = base + dk * sk + dj * sj + di;
        cv[dk][dj][di][0] = sm.bu[q];
        cv[dk][dj][di][1] = sm.bv[q];
        cv[dk][dj][di][2] = sm.bw[q];
      }
  interp_spatial<R>(cv, L, out);
}

// Wind at (lon, lat, p) and the time located by T for the active lanes;
// every thread of the block calls it.  Staged through LDS when the block's
// box fits, else gathered.
template <int F, typename R>
__device__ __forceinline__ void wind_block(const StepArgs &a, const StepLds<R> &sm, const uint16_t *s_lut, bool act,
                                           const TimeLoc &T, double lon, double lat, double p, BoxRef &ref,
                                           R out[3]) {
  Loc<R> L;
  locate_xyz<R>(a, sm.plev, sm.idp, s_lut, lon, lat, p, L);
  set_time(T, L);
  const Box b = block_box<R>(a, sm, act, L, ref);
  if (b.ok) stage_box<F, R>(a, sm, b, L);
  __syncthreads();
  if (b.ok) {
    if (act) interp_box<R>(a, sm, b, L, out);
  } else if (act) {
    Cell16<F> c;
    load_cell<F, R>(a, L, c);
    interp_cell<F, R>(a, c, L, out);
  }
}

// Midpoint advection of the block's active lanes (positions of the others
// are left alone) with the time locations of the step's start (T0) and
// midpoint (T1); every thread of the block calls it with the same ref.
template <int F, typename R>
__device__ __forceinline__ void advect_block(const StepArgs &a, const StepLds<R> &sm, const uint16_t *s_lut, bool act,
                                             const TimeLoc &T0, const TimeLoc &T1, double &lon, double &lat,
                                             double &p, BoxRef &ref) {
  auto wind = [&](int h, double x, double y, double z, R out[3]) {
    wind_block<F, R>(a, sm, s_lut, act, h ? T1 : T0, x, y, z, ref, out);
  };
  double nlon, nlat, np;
  midpoint<R>(a, lon, lat, p, wind, nlon, nlat, np);
  if (act) {
    lon = nlon;
    lat = nlat;
    p = np;
  }
}

// ---- one staging per step ------------------------------------------------------
//
// The midpoint of a step lies in or next to the cell of its start (the
// half-step displacement is far below a cell), so the box of the block's
// start cells holds most midpoint cells too, and one staging serves both
// wind evaluations of the step: the box is staged once with an FP32 pair
// per point and variable from the two time levels' values a (the earlier)
// and b (after the R16 decode and scale), and each corner is weighted in
// time when it is read, with the evaluation's own weight f, as the gather
// path's lerp, fma(f, b - a, a) in R.  For R = FP32 the pair is (a, b - a),
// one FMA per corner; for R = FP64 it is (a, b), converted when read (an
// FP64 pair would double the LDS reads, which cost more than the
// conversions).  The lanes whose midpoint cell leaves the box
// gather its records.  This saves the second box exchange, staging and pair
// of barriers at the price of the per-corner time weights.  (Widening the
// box by a cell, so that every midpoint reads LDS, staged twice the points
// and was slower than the gathers it saved.)

// Whether L's cell (all 8 corners) lies in box b.
template <typename R>
__device__ __forceinline__ bool in_box(const StepArgs &a, const Box &b, const Loc<R> &L) {
  int ci = L.i0 - b.gi;
  if (ci < 0) ci += a.nx;
  return ci <= b.bi - 2 && (unsigned)(L.j - b.j0) <= (unsigned)(b.bj - 2) &&
         (unsigned)(L.k - b.k0) <= (unsigned)(b.bk - 2);
}

// Points per pair plane: the memory of the one-time planes, or (Wide) the
// wide box region (R16: R16 storage).
template <typename R, bool Wide = false, bool R16 = false>
constexpr int pair_cap() {
  return Wide ? wide_pairs<R>(R16) : BoxCap<R>::value * (int)sizeof(R) / (int)sizeof(Pair);
}

// The three pair planes (u, v, w; point q's pair at [q]) in the box region.
template <typename R, bool Wide = false, bool R16 = false>
__device__ __forceinline__ void pair_planes(const StepLds<R> &sm, Pair *pp[3]) {
  constexpr int cap = pair_cap<R, Wide, R16>();
  Pair *base = reinterpret_cast<Pair *>(sm.bu);
  pp[0] = base;
  pp[1] = base + cap;
  pp[2] = base + 2 * cap;
}

// A point's pair from the values a, b of its two time levels: (a, b - a)
// for R = FP32, (a, b) for R = FP64.
template <typename R>
__device__ __forceinline__ Pair pair_of(float a, float b) {
  if constexpr (sizeof(R) == 8) return make_float2(a, b);
  else return make_float2(a, b - a);
}

// Stages box b's points as pairs (pair_of) of the values of time levels l
// and l1 of L (decoded and scaled for R16 storage).
template <int F, typename R>
__device__ __forceinline__ void stage_box_pairs(const StepArgs &a, Pair *const pp[3], const Box &b, const Loc<R> &L) {
  using T = typename Rec<F>::T;
  const T *lev0 = reinterpret_cast<const T *>(a.met) + (size_t)L.l * (size_t)a.level_elems;
  const T *lev1 = reinterpret_cast<const T *>(a.met) + (size_t)L.l1 * (size_t)a.level_elems;
  const int npts = b.bi * b.bj * b.bk;
  const uint32_t mi = kDivMagic.m[b.bi];
  const uint32_t mj = kDivMagic.m[b.bj];
  const float *sw0 = s_scale_win + (L.la % kScaleWin) * 3 * a.nz;
  const float *sw1 = s_scale_win + ((L.la + 1) % kScaleWin) * 3 * a.nz;
  for (int q0 = (int)threadIdx.x; q0 < npts; q0 += 2 * kBlock) {
    T r0[2], r1[2];
    int kq[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q = min(q0 + u * kBlock, npts - 1);   // a duplicate of the last point is harmless
      const int r = (int)__umulhi((uint32_t)q, mi);
      const int ii = q - r * b.bi;
      const int kk = (int)__umulhi((uint32_t)r, mj);
      const int jj = r - kk * b.bj;
      int gi = b.gi + ii;
      if (gi >= a.nx) gi -= a.nx;
      kq[u] = b.k0 + kk;
      const int off = (kq[u] * a.ny + b.j0 + jj) * a.nx + gi;   // < 2^31: nx*ny*nz is
      r0[u] = lev0[off];
      r1[u] = lev1[off];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q = min(q0 + u * kBlock, npts - 1);
      const int k = kq[u];
      float v0[3], v1[3];
      if constexpr (F == kF32) {
        v0[0] = r0[u].x; v0[1] = r0[u].y; v0[2] = r0[u].z;
        v1[0] = r1[u].x; v1[1] = r1[u].y; v1[2] = r1[u].z;
      } else {
        v0[0] = dec<F>(r0[u].x) * sw0[k]; v0[1] = dec<F>(r0[u].y) * sw0[a.nz + k];
        v0[2] = dec<F>(r0[u].z) * sw0[2 * a.nz + k];
        v1[0] = dec<F>(r1[u].x) * sw1[k]; v1[1] = dec<F>(r1[u].y) * sw1[a.nz + k];
        v1[2] = dec<F>(r1[u].z) * sw1[2 * a.nz + k];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) pp[c][q] = pair_of<R>(v0[c], v1[c]);
    }
  }
}

// The wind at L from the pair planes of box b: each corner's pair weighted
// in time with L.ft (the lerp of the gather path), then the spatial
// interpolation (interp_spatial's operations; for R = FP32 one variable at
// a time, so that only one variable's pairs are held at once).
template <typename R>
__device__ __forceinline__ void interp_pairs(const StepArgs &a, Pair *const pp[3], const Box &b, const Loc<R> &L,
                                             R out[3]) {
  int ci = L.i0 - b.gi;
  if (ci < 0) ci += a.nx;
  const int sj = b.bi, sk = b.bi * b.bj;
  const int base = (L.k - b.k0) * sk + (L.j - b.j0) * sj + ci;
  if constexpr (sizeof(R) == 8) {
    R cv[2][2][2][3];
#pragma unroll
    for (int dk = 0; dk < 2; ++dk)
#pragma unroll
      for (int dj = 0; dj < 2; ++dj)
#pragma unroll
        for (int di = 0; di < 2; ++di) {
          const int q = base + dk * sk + dj * sj + di;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float2 v = pp[c][q];
            cv[dk][dj][di][c] = lerp((R)v.x, (R)v.y, L.ft);
          }
        }
    interp_spatial<R>(cv, L, out);
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      R cv[2][2][2];
#pragma unroll
      for (int dk = 0; dk < 2; ++dk)
#pragma unroll
        for (int dj = 0; dj < 2; ++dj)
#pragma unroll
          for (int di = 0; di < 2; ++di) {
            const float2 v = pp[c][base + dk * sk + dj * sj + di];
            cv[dk][dj][di] = fma(L.ft, v.y, v.x);
          }
      R yk[2];
#pragma unroll
      for (int dk = 0; dk < 2; ++dk) {
        const R x0 = lerp(cv[dk][0][0], cv[dk][0][1], L.fx);
        const R x1 = lerp(cv[dk][1][0], cv[dk][1][1], L.fx);
        yk[dk] = lerp(x0, x1, L.fy);
      }
      out[c] = lerp(yk[0], yk[1], L.fz);
    }
  }
}

// advect_block with one box exchange and one staging per step: the box of
// the start cells is staged as pairs; the start winds read it, and so do
// the midpoint winds of the lanes whose midpoint cell lies in it when the
// midpoint time uses the start's time-level pair; the other lanes gather.
// Every thread of the block calls it with the same ref; the winds are
// those of advect_block bit for bit.
template <int F, typename R>
__device__ __forceinline__ void advect_block_one(const StepArgs &a, const StepLds<R> &sm, const uint16_t *s_lut,
                                                 bool act, const TimeLoc &T0, const TimeLoc &T1, double &lon,
                                                 double &lat, double &p, BoxRef &ref) {
  Pair *pp[3];
  pair_planes<R, true>(sm, pp);
  const bool same = T0.l == T1.l && T0.l1 == T1.l1 && T0.la == T1.la;   // uniform
  Box s;
  s.ok = false;
  auto wind = [&](int h, double x, double y, double z, R out[3]) {
    Loc<R> L;
    locate_xyz<R>(a, sm.plev, sm.idp, s_lut, x, y, z, L);
    if (h == 0) {
      set_time(T0, L);
      s = block_box<R>(a, sm, act, L, ref);
      s.ok = s.ok && s.bi * s.bj * s.bk <= pair_cap<R, true>();
      if (s.ok) stage_box_pairs<F, R>(a, pp, s, L);
      __syncthreads();
      if (!act) return;
      if (s.ok) {
        interp_pairs<R>(a, pp, s, L, out);
        return;
      }
    } else {
      set_time(T1, L);
      if (!act) return;
      if (same && s.ok && in_box(a, s, L)) {
        interp_pairs<R>(a, pp, s, L, out);
        return;
      }
    }
    Cell16<F> c;
    load_cell<F, R>(a, L, c);
    interp_cell<F, R>(a, c, L, out);
  };
  double nlon, nlat, np;
  midpoint<R>(a, lon, lat, p, wind, nlon, nlat, np);
  if (act) {
    lon = nlon;
    lat = nlat;
    p = np;
  }
}

// One pass of stage_box_pairs over points q0 and q0 + kBlock (each clamped
// to the box's last point), with mid() run between the loads and their use.
template <int F, typename R, typename Mid>
__device__ __forceinline__ void pair_pass(const StepArgs &a, Pair *const pp[3], const Box &b, const Loc<R> &L,
                                          int q0, Mid &&mid) {
  using T = typename Rec<F>::T;
  const T *lev0 = reinterpret_cast<const T *>(a.met) + (size_t)L.l * (size_t)a.level_elems;
  const T *lev1 = reinterpret_cast<const T *>(a.met) + (size_t)L.l1 * (size_t)a.level_elems;
  const int npts = b.bi * b.bj * b.bk;
  const uint32_t mi = kDivMagic.m[b.bi];
  const uint32_t mj = kDivMagic.m[b.bj];
  const float *sw0 = s_scale_win + (L.la % kScaleWin) * 3 * a.nz;
  const float *sw1 = s_scale_win + ((L.la + 1) % kScaleWin) * 3 * a.nz;
  T r0[2], r1[2];
  int kq[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int q = min(q0 + u * kBlock, npts - 1);
    const int r = (int)__umulhi((uint32_t)q, mi);
    const int ii = q - r * b.bi;
    const int kk = (int)__umulhi((uint32_t)r, mj);
    const int jj = r - kk * b.bj;
    int gi = b.gi + ii;
    if (gi >= a.nx) gi -= a.nx;
    kq[u] = b.k0 + kk;
    const int off = (kq[u] * a.ny + b.j0 + jj) * a.nx + gi;   // < 2^31: nx*ny*nz is
    r0[u] = lev0[off];
    r1[u] = lev1[off];
  }
  mid();
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int q = min(q0 + u * kBlock, npts - 1);
    const int k = kq[u];
    float v0[3], v1[3];
    if constexpr (F == kF32) {
      v0[0] = r0[u].x; v0[1] = r0[u].y; v0[2] = r0[u].z;
      v1[0] = r1[u].x; v1[1] = r1[u].y; v1[2] = r1[u].z;
    } else {
      v0[0] = dec<F>(r0[u].x) * sw0[k]; v0[1] = dec<F>(r0[u].y) * sw0[a.nz + k];
      v0[2] = dec<F>(r0[u].z) * sw0[2 * a.nz + k];
      v1[0] = dec<F>(r1[u].x) * sw1[k]; v1[1] = dec<F>(r1[u].y) * sw1[a.nz + k];
      v1[2] = dec<F>(r1[u].z) * sw1[2 * a.nz + k];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) pp[c][q] = pair_of<R>(v0[c], v1[c]);
  }
}

// stage_box_pairs with fill() run once in every thread between the first
// pass's loads and their use (the first pass runs in every thread: npts >= 8,
// a thread past the box rewrites the box's last point).
template <int F, typename R, typename Fill>
__device__ __forceinline__ void stage_box_pairs_fill(const StepArgs &a, Pair *const pp[3], const Box &b,
                                                     const Loc<R> &L, Fill &&fill) {
  const int npts = b.bi * b.bj * b.bk;
  pair_pass<F, R>(a, pp, b, L, (int)threadIdx.x, fill);
  for (int q0 = (int)threadIdx.x + 2 * kBlock; q0 < npts; q0 += 2 * kBlock) pair_pass<F, R>(a, pp, b, L, q0, [] {});
}

// advect_block_one with the box region of pair_cap<R, Wide>() points and
// fill() run once in every thread while the staging's first loads are in
// flight (or before the gathers when nothing is staged).
template <int F, typename R, bool Wide, typename Fill>
__device__ __forceinline__ void advect_block_one_fill(const StepArgs &a, const StepLds<R> &sm, const uint16_t *s_lut,
                                                      bool act, const TimeLoc &T0, const TimeLoc &T1, double &lon,
                                                      double &lat, double &p, BoxRef &ref, Fill &&fill) {
  Pair *pp[3];
  pair_planes<R, Wide, F != kF32>(sm, pp);
  constexpr int cap = pair_cap<R, Wide, F != kF32>();
  const bool same = T0.l == T1.l && T0.l1 == T1.l1 && T0.la == T1.la;   // uniform
  Box s;
  s.ok = false;
  auto wind = [&](int h, double x, double y, double z, R out[3]) {
    Loc<R> L;
    locate_xyz<R>(a, sm.plev, sm.idp, s_lut, x, y, z, L);
    if (h == 0) {
      set_time(T0, L);
      s = block_box<R>(a, sm, act, L, ref);
      s.ok = s.ok && s.bi * s.bj * s.bk <= cap;
      if (s.ok) stage_box_pairs_fill<F, R>(a, pp, s, L, fill);
      else fill();
      __syncthreads();
      if (!act) return;
      if (s.ok) {
        interp_pairs<R>(a, pp, s, L, out);
        return;
      }
    } else {
      set_time(T1, L);
      if (!act) return;
      if (same && s.ok && in_box(a, s, L)) {
        interp_pairs<R>(a, pp, s, L, out);
        return;
      }
    }
    Cell16<F> c;
    load_cell<F, R>(a, L, c);
    interp_cell<F, R>(a, c, L, out);
  };
  double nlon, nlat, np;
  midpoint<R>(a, lon, lat, p, wind, nlon, nlat, np);
  if (act) {
    lon = nlon;
    lat = nlat;
    p = np;
  }
}

}  // namespace mpt
