// mpt_device.h -- device building blocks of the particle time step (gfx950).
//
// Internal to libmpt.  Everything here is compiled with -ffp-contract=off:
// fused multiply-adds appear only where written as fma(), so the fused
// multi-step kernel and the split advect / diffuse kernels execute the same
// floating-point operations in the same order (bitwise-equal results).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

#include "mpt_math.h"

namespace mpt {

// ---- constants of the method ------------------------------------------------
constexpr double kPi = 3.14159265358979323846;
constexpr double kREarth = 6371000.0;                 // m
constexpr double kH0 = 7000.0;                        // scale height, dz -> dp [m]
constexpr double kDeg = 180.0 / (kPi * kREarth);      // metres -> degrees of arc
constexpr double kG = 9.80665;                        // m s^-2 (box air mass, settling)
constexpr double kRd = 287.058;                       // gas constant of dry air [J/(kg K)]
constexpr int kMaxLevels = 512;                       // LDS level table capacity
constexpr int kLutBins = 4096;                        // level lookup bins over log2(p)
constexpr int kBlock = 256;                           // 4 wave64 per block
constexpr int kXcds = 8;                              // MI355X: 8 XCDs, 32 CUs each

enum : uint32_t { kAdvect = 1u, kTurb = 2u, kMeso = 4u, kConv = 8u, kSedi = 16u };
enum FieldKind { kF32 = 0, kBF16 = 1, kF16 = 2 };

// Arguments of the step kernels, passed by value.
struct StepArgs {
  double *lon, *lat, *p;
  const uint32_t *id;
  void *up, *vp, *wp;
  const uint16_t *scen;        // may be null
  const int32_t *release;      // per scenario, device; null when scen is null
  int64_t n;

  const void *met;             // packed levels, ring slot s at met + s*level_elems records
  int64_t level_elems;         // nx*ny*nz
  // Spread of the 16 values of each cell per variable, for the level pair
  // whose earlier level sits in ring slot s, at sig + s*level_elems records
  // (cell (k, j, i) at (k*ny + j)*nx + i): {su, sv, sw, 0} as double (FP64
  // arithmetic) or float; null without mesoscale diffusion.
  const void *sig;
  const float *scales;         // [nt][3][nz] (R16 storage)
  const double *plev;          // [nz] device
  const double *inv_dp;        // [nz-1] 1 / (plev[k] - plev[k+1])
  const uint16_t *lut;         // [kLutBins] level lower bound per log2(p) bin
  float lut_lo, lut_scale;     // bin = (log2(p) - lut_lo) * lut_scale
  int nx, ny, nz, nt;
  double lon0, inv_dlon, lat0, inv_dlat, lat_hi, p_top, p_bot;
  double t_met0, dt_met, inv_dt_met;

  double dt, t_start;
  double sig_h, sig_z;         // sqrt(2 D dt) [m]
  double r_ar, rs_fh, rs_fv;   // AR(1): r, sqrt(1-r^2)*fh, sqrt(1-r^2)*fv
  double cos_cap;              // cos(89.999 deg)
  uint64_t seed;
  uint32_t step0;              // first step (added to *step_dev when that is set)
  int32_t nsteps;
  uint32_t flags;
  int32_t nblk;                // logical blocks
  int32_t per_xcd;             // logical blocks per XCD

  // Step index in device memory (replayable graphs); null = step0 alone.
  const uint32_t *step_dev;
  // Persistent mode (scenario runs right after a sort): parcels are ordered
  // active-by-tile, then pending scenarios by release rank, then non-finite;
  // the kernel walks only the prefix of parcels released by the launch's
  // last step: offsets[ntiles + r], r = #(rel_sorted <= last step).
  int32_t persistent;
  int32_t nscen;
  uint32_t ntiles;
  const uint32_t *offsets;     // exclusive scan of the last sort's histogram
  const int32_t *rel_sorted;   // release steps in ascending order [nscen]
  // Index-list mode: advance only parcels index[0 .. *index_count).
  const uint32_t *index;
  const uint32_t *index_count;
  // Resident met levels: absolute index of the oldest and its ring slot.
  int32_t lev_first, slot_first;
  // Convection and sedimentation: surface records {cape, pel, ps, 0} per
  // (ring slot, j, i); temperature scales per (ring slot, level) for R16
  // storage; CAPE threshold, particle radius and density.
  const float4 *sfc;
  const float *t_scales;
  double conv_cape, sedi_r, sedi_rho;
  // Sort keys of the final positions (block launches only; null: none).
  // Device memory, read after the step loop, so its fields hold no scalar
  // registers during it.
  const struct SortKeyArgs *sk;
  // Deferred sort (block launches only; null: none): parcel i of the sorted
  // order is read from index src[i] of the arrays above and its whole state
  // (position, id, mesoscale state) is written to index i of the *_o
  // arrays, for every parcel, moved or not.
  const uint32_t *src;
  double *lon_o, *lat_o, *p_o;
  uint32_t *id_o;
  void *up_o, *vp_o, *wp_o;
};

// Where a launch leaves the sort keys: tile key and rank within the key
// from run-aggregated atomics on the sort's spread counters (key k at
// (k % 16) * spread_s + k / 16).
struct SortKeyArgs {
  uint32_t *keys, *ranks, *spread;
  uint32_t spread_s, ntx, nty, nkeys;
};

// Map the hardware block index to a logical block so that each XCD walks a
// contiguous range of (sorted) parcels: hardware dispatch is round-robin
// over the XCDs, so block b runs on XCD b % 8.
__device__ __forceinline__ int logical_block(int b, int per_xcd) {
  return (b % kXcds) * per_xcd + b / kXcds;
}

// ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) ----------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

template <typename R> struct Math;

template <> struct Math<double> {
  // ((x >> 8) + 1/2) / 2^24 and twice that, each one exact FMA
  static __device__ __forceinline__ double uni(uint32_t x) {
    return fma((double)(x >> 8), 0x1p-24, 0x1p-25);
  }
  static __device__ __forceinline__ double uni2(uint32_t x) {
    return fma((double)(x >> 8), 0x1p-23, 0x1p-24);
  }
  // ln of a uniform in (0, 1): always a positive normal number
  static __device__ __forceinline__ double log_(double x) { return m64::ln_pos(x); }
  // non-negative arguments: Box-Muller radii, variances (0 when a cell's
  // values are equal), temperatures; below 2^-900 the root is taken as 0
  static __device__ __forceinline__ double sqrt_(double x) {
    return x > 0x1p-900 ? m64::sqrt_pos(x) : 0.0;
  }
  static __device__ __forceinline__ double exp_(double x) { return exp(x); }
  // sin(pi x), cos(pi x) for x in [0, 2] (twice a uniform)
  static __device__ __forceinline__ void sincospi_(double x, double *s, double *c) {
    m64::sincospi_02(x, s, c);
  }
  static __device__ __forceinline__ double cospi_(double x) { return m64::cospi_02(x); }
  // 1/x for x in [cos 89.999 deg, 1]: hardware estimate + two Newton steps
  // (error squared per step, final error at the rounding level)
  static __device__ __forceinline__ double rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
  }
};

template <> struct Math<float> {
  static __device__ __forceinline__ float uni(uint32_t x) {
    return ((float)(x >> 8) + 0.5f) * (1.0f / 16777216.0f);
  }
  // hardware log2 and square root (within 1 ulp, no denormal scaling): the
  // arguments are uniforms >= 2^-25, Box-Muller radii and spreads (the
  // spreads' zero maps to zero)
  static __device__ __forceinline__ float log_(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
  static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
  static __device__ __forceinline__ float exp_(float x) { return __expf(x); }
  static __device__ __forceinline__ void sincospi_(float x, float *s, float *c) {
    __sincosf(x * (float)kPi, s, c);
  }
  static __device__ __forceinline__ float cospi_(float x) { return __cosf(x * (float)kPi); }
  // hardware reciprocal (within 1 ulp): x in [cos 89.999 deg, 1]
  static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
};

// Three standard normals for (id, step, purpose): Box-Muller on one Philox
// block, uniforms ((x >> 8) + 1/2) / 2^24.
template <typename R>
__device__ __forceinline__ void normals3(uint64_t seed, uint32_t id, uint32_t step, uint32_t purpose,
                                         R xi[3]) {
  uint32_t x[4];
  // The key words are tied to the step (an empty asm that takes the step as
  // input), so the nine round keys are formed on the scalar unit at each
  // draw instead of being hoisted out of the step loop, where they would be
  // spilled to vector lanes and read back every step.
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  asm("" : "+s"(k0), "+s"(k1) : "s"(step));
  philox4x32_10(id, step, purpose, 0u, k0, k1, x);
  if constexpr (sizeof(R) == 8) {
    // the angles' 2 u1 and 2 u3 formed directly (one exact FMA each)
    const R u0 = Math<R>::uni(x[0]), t1 = Math<R>::uni2(x[1]);
    const R u2 = Math<R>::uni(x[2]), t3 = Math<R>::uni2(x[3]);
    const R r0 = Math<R>::sqrt_((R)-2 * Math<R>::log_(u0));
    const R r1 = Math<R>::sqrt_((R)-2 * Math<R>::log_(u2));
    R s1, c1;
    Math<R>::sincospi_(t1, &s1, &c1);           // angle 2 pi u1
    xi[0] = r0 * c1;
    xi[1] = r0 * s1;
    xi[2] = r1 * Math<R>::cospi_(t3);
  } else {
    const R u0 = Math<R>::uni(x[0]), u1 = Math<R>::uni(x[1]);
    const R u2 = Math<R>::uni(x[2]), u3 = Math<R>::uni(x[3]);
    const R r0 = Math<R>::sqrt_((R)-2 * Math<R>::log_(u0));
    const R r1 = Math<R>::sqrt_((R)-2 * Math<R>::log_(u2));
    R s1, c1;
    Math<R>::sincospi_((R)2 * u1, &s1, &c1);    // angle 2 pi u1
    xi[0] = r0 * c1;
    xi[1] = r0 * s1;
    xi[2] = r1 * Math<R>::cospi_((R)2 * u3);
  }
}

// ---- field records -----------------------------------------------------------
template <int F> struct Rec;
template <> struct Rec<kF32> { using T = float4; };
template <> struct Rec<kBF16> { using T = ushort4; };
template <> struct Rec<kF16> { using T = ushort4; };

template <int F> __device__ __forceinline__ float dec(unsigned short q);
template <> __device__ __forceinline__ float dec<kBF16>(unsigned short q) {
  return __uint_as_float((uint32_t)q << 16);
}
template <> __device__ __forceinline__ float dec<kF16>(unsigned short q) {
  return (float)__builtin_bit_cast(_Float16, q);
}

// The three stored values of one grid point as R (decoded with the scales of
// its (level, time level) for R16 storage).
template <int F, typename R>
struct Fetch {
  static __device__ __forceinline__ void get(const typename Rec<F>::T &v, const float *sc, R o[3]) {
    o[0] = (R)(dec<F>(v.x) * sc[0]);
    o[1] = (R)(dec<F>(v.y) * sc[1]);
    o[2] = (R)(dec<F>(v.z) * sc[2]);
  }
};
template <typename R>
struct Fetch<kF32, R> {
  static __device__ __forceinline__ void get(const float4 &v, const float *, R o[3]) {
    o[0] = (R)v.x;
    o[1] = (R)v.y;
    o[2] = (R)v.z;
  }
};

// ---- locate ----------------------------------------------------------------------
template <typename R>
struct Loc {
  int i0, i1, j, k;
  int l, l1;            // storage slots of the earlier and the later time level
  int la;               // absolute index of the earlier time level
  R fx, fy, fz, ft;
};

// Level bracket: k = largest index <= nz-2 with plev[k] >= pc.  A bin of
// log2(pc) (FP32) gives a starting k from the LDS lookup table; the FP64
// comparisons that follow make the result exact whatever bin FP32 picked.
__device__ __forceinline__ int level_index(const StepArgs &a, const double *s_plev,
                                           const uint16_t *s_lut, double pc) {
  int b = (int)((__log2f((float)pc) - a.lut_lo) * a.lut_scale);
  b = min(max(b, 0), kLutBins - 1);
  int k = s_lut[b];
  while (k < a.nz - 2 && s_plev[k + 1] >= pc) ++k;
  while (k > 0 && s_plev[k] < pc) --k;
  return k;
}

// Horizontal and vertical part of the cell location.  Longitude periodic,
// latitude and pressure clamped; k from level_index.
template <typename R>
__device__ __forceinline__ void locate_xyz(const StepArgs &a, const double *s_plev,
                                           const double *s_idp, const uint16_t *s_lut, double lon,
                                           double lat, double p, Loc<R> &L) {
  const double lam = lon - 360.0 * floor((lon - a.lon0) * (1.0 / 360.0));
  const double x = (lam - a.lon0) * a.inv_dlon;
  const double xf = floor(x);
  int i0 = (int)xf;
  if (i0 >= a.nx) i0 -= a.nx;
  if (i0 < 0) i0 += a.nx;
  L.i0 = i0;
  L.i1 = (i0 + 1 == a.nx) ? 0 : i0 + 1;
  L.fx = (R)(x - xf);

  const double phi = fmin(fmax(lat, a.lat0), a.lat_hi);
  const double y = (phi - a.lat0) * a.inv_dlat;
  int j = (int)floor(y);
  j = min(max(j, 0), a.ny - 2);
  L.j = j;
  L.fy = (R)(y - (double)j);

  const double pc = fmin(fmax(p, a.p_top), a.p_bot);
  // level_index with the table's guess k0 and the levels and inverse
  // spacings around it read together (one LDS round trip after the
  // table's), which settles the usual one step up without another; further
  // steps (rare) walk on as level_index does.  Same k.
  int b = (int)((__log2f((float)pc) - a.lut_lo) * a.lut_scale);
  b = min(max(b, 0), kLutBins - 1);
  const int k0 = s_lut[b];
  const int k1 = min(k0 + 1, a.nz - 1);
  const double p0 = s_plev[k0], p1 = s_plev[k1], d0 = s_idp[k0], d1 = s_idp[k1];
  int k = k0;
  double pk = p0, dk = d0;
  if (k0 < a.nz - 2 && p1 >= pc) {
    k = k1;
    pk = p1;
    dk = d1;
    if (k < a.nz - 2 && s_plev[k + 1] >= pc) {
      while (k < a.nz - 2 && s_plev[k + 1] >= pc) ++k;
      pk = s_plev[k];
      dk = s_idp[k];
    }
  } else if (k0 > 0 && p0 < pc) {
    while (k > 0 && s_plev[k] < pc) --k;
    pk = s_plev[k];
    dk = s_idp[k];
  }
  L.k = k;
  L.fz = (R)((pk - pc) * dk);
}

// locate_xyz for tables read from global memory (kernels that visit each
// parcel once and do not stage them in LDS).  The level table's guess k0 and
// the four levels and inverse spacings around it are loaded together, which
// settles up to two steps either way without another round trip (further
// steps, rare, walk on); same cell and weights as locate_xyz.
template <typename R>
__device__ __forceinline__ void locate_xyz_g(const StepArgs &a, double lon, double lat, double p, Loc<R> &L) {
  const double lam = lon - 360.0 * floor((lon - a.lon0) * (1.0 / 360.0));
  const double x = (lam - a.lon0) * a.inv_dlon;
  const double xf = floor(x);
  int i0 = (int)xf;
  if (i0 >= a.nx) i0 -= a.nx;
  if (i0 < 0) i0 += a.nx;
  L.i0 = i0;
  L.i1 = (i0 + 1 == a.nx) ? 0 : i0 + 1;
  L.fx = (R)(x - xf);

  const double phi = fmin(fmax(lat, a.lat0), a.lat_hi);
  const double y = (phi - a.lat0) * a.inv_dlat;
  int j = (int)floor(y);
  j = min(max(j, 0), a.ny - 2);
  L.j = j;
  L.fy = (R)(y - (double)j);

  const double pc = fmin(fmax(p, a.p_top), a.p_bot);
  int b = (int)((__log2f((float)pc) - a.lut_lo) * a.lut_scale);
  b = min(max(b, 0), kLutBins - 1);
  const int k0 = a.lut[b];
  const int top = a.nz - 2;
  const int km = max(k0 - 1, 0), k1 = min(k0 + 1, a.nz - 1), k2 = min(k0 + 2, a.nz - 1);
  const double pm = a.plev[km], p0 = a.plev[k0], p1 = a.plev[k1], p2 = a.plev[k2];
  const double dm = a.inv_dp[km], d0 = a.inv_dp[k0], d1 = a.inv_dp[k1], d2 = a.inv_dp[k2];
  int k = k0;
  double pk = p0, dk = d0;
  if (k < top && p1 >= pc) {
    k = k0 + 1; pk = p1; dk = d1;
    if (k < top && p2 >= pc) {
      k = k0 + 2; pk = p2; dk = d2;
      while (k < top && a.plev[k + 1] >= pc) ++k;
      if (k > k0 + 2) { pk = a.plev[k]; dk = a.inv_dp[k]; }
    }
  } else if (k > 0 && p0 < pc) {
    k = k0 - 1; pk = pm; dk = dm;
    if (k > 0 && pm < pc) {
      --k;
      while (k > 0 && a.plev[k] < pc) --k;
      pk = a.plev[k]; dk = a.inv_dp[k];
    }
  }
  L.k = k;
  L.fz = (R)((pk - pc) * dk);
}

// Time-level pair bracketing t and the weight of the later level.  The
// resident levels are lev_first .. lev_first + nt - 1 (absolute indices,
// level L at t_met0 + L dt_met), stored in a ring of nt slots starting at
// slot_first; the pair is clamped to the resident window.
__device__ __forceinline__ int met_level(const StepArgs &a, double t) {
  double tl = floor((t - a.t_met0) * a.inv_dt_met);
  int l = (int)tl;
  if (tl < (double)a.lev_first) l = a.lev_first;
  if (l > a.lev_first + a.nt - 2) l = a.lev_first + a.nt - 2;
  return l;
}

// The time part of a location: storage slots of the level pair, absolute
// index of the earlier level, weight of the later one.
struct TimeLoc {
  int l, l1, la;
  double ft;
};

__device__ __forceinline__ TimeLoc time_loc(const StepArgs &a, double t) {
  TimeLoc T;
  const int l = met_level(a, t);
  T.la = l;
  int s0 = a.slot_first + (l - a.lev_first);
  if (s0 >= a.nt) s0 -= a.nt;
  T.l = s0;
  T.l1 = s0 + 1 == a.nt ? 0 : s0 + 1;
  T.ft = (t - (a.t_met0 + (double)l * a.dt_met)) * a.inv_dt_met;
  return T;
}

template <typename R>
__device__ __forceinline__ void set_time(const TimeLoc &T, Loc<R> &L) {
  L.la = T.la;
  L.l = T.l;
  L.l1 = T.l1;
  L.ft = (R)T.ft;
}

template <typename R>
__device__ __forceinline__ void locate_t(const StepArgs &a, double t, Loc<R> &L) {
  set_time(time_loc(a, t), L);
}

// Time locations of a run of steps held across the lanes of a wave: lane e
// has that of step step_base + e / 2 at its start (e even) or at its
// midpoint, start + dt/2 (e odd).  time_at reads entry e (uniform) back into
// scalar registers; 32 steps per table.
constexpr int kTimeTableSteps = 32;
struct TimeTable {
  TimeLoc v;
};

__device__ __forceinline__ TimeTable time_table(const StepArgs &a, uint32_t step_base) {
  const int e = (int)(threadIdx.x & 63);
  double t = a.t_start + (double)(step_base + (uint32_t)(e >> 1)) * a.dt;
  if (e & 1) t = t + 0.5 * a.dt;
  return TimeTable{time_loc(a, t)};
}

__device__ __forceinline__ TimeLoc time_at(const TimeTable &tt, int e) {
  TimeLoc T;
  T.l = __builtin_amdgcn_readlane(tt.v.l, e);
  T.l1 = __builtin_amdgcn_readlane(tt.v.l1, e);
  T.la = __builtin_amdgcn_readlane(tt.v.la, e);
  const uint64_t bits = __double_as_longlong(tt.v.ft);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)bits, e);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(bits >> 32), e);
  T.ft = __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
  return T;
}

template <typename R>
__device__ __forceinline__ R lerp(R a, R b, R f) { return fma(f, b - a, a); }

// The 16 records of a cell: 2 time levels x 2 levels x 2 rows x 2 columns.
template <int F>
struct Cell16 {
  typename Rec<F>::T r[2][2][2][2];   // [dl][dk][dj][di]
};

// Two consecutive 8-byte records read by one 16-byte load.
struct __attribute__((aligned(8))) RecPair8 {
  ushort4 a, b;
};

// 16-byte records: one load per corner.  8-byte records: the two corners of
// a row are consecutive in memory except across the periodic seam, so one
// 16-byte load fetches both (half the gather instructions); a parcel on the
// seam (i0 = nx - 1, i1 = 0) loads the pair ending at i0 and record 0.
// The wave forms the addresses and issues the loads at raised priority (the
// step's callers raise it already before the locate), so its gathers are in
// flight sooner while the other waves of the SIMD compute; it drops back
// once they are issued.
template <int F, typename R>
__device__ __forceinline__ void load_cell(const StepArgs &a, const Loc<R> &L, Cell16<F> &c) {
  using T = typename Rec<F>::T;
  __builtin_amdgcn_s_setprio(2);
  const T *base = reinterpret_cast<const T *>(a.met);
  const int nxy = a.nx * a.ny;
  const int r0 = L.k * nxy + L.j * a.nx;
  const bool seam = L.i1 < L.i0;
  const int ip = seam ? L.i0 - 1 : L.i0;
#pragma unroll
  for (int dl = 0; dl < 2; ++dl) {
    const T *lev = base + (int64_t)(dl ? L.l1 : L.l) * a.level_elems;
#pragma unroll
    for (int dk = 0; dk < 2; ++dk)
#pragma unroll
      for (int dj = 0; dj < 2; ++dj) {
        const T *row = lev + r0 + dk * nxy + dj * a.nx;
        if constexpr (F == kF32) {
          c.r[dl][dk][dj][0] = row[L.i0];
          c.r[dl][dk][dj][1] = row[L.i1];
        } else {
          const RecPair8 q = *reinterpret_cast<const RecPair8 *>(row + ip);
          c.r[dl][dk][dj][0] = q.a;
          c.r[dl][dk][dj][1] = q.b;
          if (seam) {
            c.r[dl][dk][dj][0] = q.b;
            c.r[dl][dk][dj][1] = row[0];
          }
        }
      }
  }
  __builtin_amdgcn_s_setprio(0);
}

// R16 storage: the step kernels keep the per-level scales of the met time
// levels a launch reads in LDS (dynamic shared memory, kScaleWin x 3 x nz
// floats): absolute level L at window row L % kScaleWin.  A launch whose
// times span less than one met interval reads at most three consecutive
// levels (the pair of its first time, and the next one); the host keeps
// launches of R16 storage that short.
constexpr int kScaleWin = 3;
extern __shared__ float s_scale_win[];

// Fills the window with the scales of levels lev .. lev + 2 (those that are
// resident), lev being the earlier level of the launch's first time.  All
// threads of the block call it; a barrier must follow before any read.
__device__ __forceinline__ void stage_scale_window(const StepArgs &a, int lev) {
  const int row = 3 * a.nz;
  for (int q = threadIdx.x; q < kScaleWin * row; q += kBlock) {
    const int d = q / row, r = q - d * row;
    const int L = lev + d;
    if (L > a.lev_first + a.nt - 1) continue;
    int slot = a.slot_first + (L - a.lev_first);
    if (slot >= a.nt) slot -= a.nt;
    s_scale_win[(L % kScaleWin) * row + r] = a.scales[(int64_t)slot * row + r];
  }
}

// Scales of the (time level, level) slabs a cell touches (R16 storage:
// from the LDS window).
template <int F, typename R>
__device__ __forceinline__ void cell_scales(const StepArgs &a, const Loc<R> &L, float sc[2][2][3]) {
#pragma unroll
  for (int dl = 0; dl < 2; ++dl)
#pragma unroll
    for (int dk = 0; dk < 2; ++dk) {
      if (F == kF32) {
        sc[dl][dk][0] = sc[dl][dk][1] = sc[dl][dk][2] = 1.0f;
      } else {
        const float *s = s_scale_win + ((L.la + dl) % kScaleWin) * 3 * a.nz + (L.k + dk);
        sc[dl][dk][0] = s[0];
        sc[dl][dk][1] = s[a.nz];
        sc[dl][dk][2] = s[2 * a.nz];
      }
    }
}

// Quadrilinear interpolation, the time weight applied first at each of the
// 8 corners, then along lon, lat and p.  Equal to interpolating in space at
// both time levels and then in time (multilinear), up to rounding.  The
// staged path (mpt_stage.h) forms the same time-weighted corner values once
// per grid point and then runs the same spatial part, so both paths give the
// same bits.
template <typename R>
__device__ __forceinline__ void interp_spatial(const R cv[2][2][2][3], const Loc<R> &L, R out[3]) {
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    R yk[2];
#pragma unroll
    for (int dk = 0; dk < 2; ++dk) {
      const R x0 = lerp(cv[dk][0][0][q], cv[dk][0][1][q], L.fx);
      const R x1 = lerp(cv[dk][1][0][q], cv[dk][1][1][q], L.fx);
      yk[dk] = lerp(x0, x1, L.fy);
    }
    out[q] = lerp(yk[0], yk[1], L.fz);
  }
}

template <int F, typename R>
__device__ __forceinline__ void interp_cell(const StepArgs &a, const Cell16<F> &c, const Loc<R> &L,
                                            R out[3]) {
  float sc[2][2][3];
  cell_scales<F, R>(a, L, sc);
  R cv[2][2][2][3];   // [dk][dj][di][var], time-interpolated
#pragma unroll
  for (int dk = 0; dk < 2; ++dk)
#pragma unroll
    for (int dj = 0; dj < 2; ++dj)
#pragma unroll
      for (int di = 0; di < 2; ++di) {
        R v0[3], v1[3];
        Fetch<F, R>::get(c.r[0][dk][dj][di], sc[0][dk], v0);
        Fetch<F, R>::get(c.r[1][dk][dj][di], sc[1][dk], v1);
#pragma unroll
        for (int q = 0; q < 3; ++q) cv[dk][dj][di][q] = lerp(v0[q], v1[q], L.ft);
      }
  interp_spatial<R>(cv, L, out);
}

// cos(lat) floored at cos(89.999 deg).  The value must keep its relative
// accuracy near the poles, where 1/cos(lat) scales the longitude increments
// and a cosine of a rounded angle has an absolute error.  FP64: the sine of
// the co-latitude by its minimax polynomial.  FP32: within 0.5 rad of a pole the
// sine of the co-latitude (formed in FP64) by its series to x^7 (relative
// error below 1e-9), elsewhere (cos >= 0.48) the hardware cosine.
template <typename R>
__device__ __forceinline__ R cos_floor(const StepArgs &a, double lat) {
  R c;
  if constexpr (sizeof(R) == 8) {
    c = m64::cos_lat_deg(lat);
  } else {
    const float x = (float)((90.0 - fabs(lat)) * (kPi / 180.0));
    if (x < 0.5f) {
      const float x2 = x * x;
      c = (R)(x * (1.0f - x2 * (1.0f / 6.0f) * (1.0f - x2 * (1.0f / 20.0f) * (1.0f - x2 * (1.0f / 42.0f)))));
    } else {
      c = (R)__cosf((float)(lat * (kPi / 180.0)));
    }
  }
  return c > (R)a.cos_cap ? c : (R)a.cos_cap;
}

// ---- modules -----------------------------------------------------------------------

// Explicit midpoint: x_mid = x + dt/2 f(x, t); x' = x + dt f(x_mid, t + dt/2),
// f = (u / (R cos lat), v / R, omega) in degrees and hPa per second.  The
// wind at a point comes from `wind(h, lon, lat, p, out)`, at the step's time
// t (h = 0) or at t + dt/2 (h = 1); the new position goes to (nlon, nlat,
// np).
template <typename R, typename Wind>
__device__ __forceinline__ void midpoint(const StepArgs &a, double lon, double lat, double p, Wind &&wind,
                                         double &nlon, double &nlat, double &np) {
  R w0[3], w1[3];
  wind(0, lon, lat, p, w0);
  const R hdt = (R)(0.5 * a.dt);
  const R kdeg = (R)kDeg;
  const R d0lon = w0[0] * kdeg * Math<R>::rcp(cos_floor<R>(a, lat));
  const R d0lat = w0[1] * kdeg;
  const double lonm = lon + (double)(hdt * d0lon);
  const double latm = lat + (double)(hdt * d0lat);
  const double pm = p + (double)(hdt * w0[2]);
  wind(1, lonm, latm, pm, w1);
  const R fdt = (R)a.dt;
  const R d1lon = w1[0] * kdeg * Math<R>::rcp(cos_floor<R>(a, latm));
  const R d1lat = w1[1] * kdeg;
  nlon = lon + (double)(fdt * d1lon);
  nlat = lat + (double)(fdt * d1lat);
  np = p + (double)(fdt * w1[2]);
}

// Midpoint advection with each wind gathered from global memory.
template <int F, typename R>
__device__ __forceinline__ void advect(const StepArgs &a, const double *s_plev, const double *s_idp,
                                       const uint16_t *s_lut, double t, double &lon, double &lat,
                                       double &p) {
  auto wind = [&](int h, double x, double y, double z, R out[3]) {
    Cell16<F> c;
    Loc<R> L;
    __builtin_amdgcn_s_setprio(2);   // locate and gather at raised priority
    locate_xyz<R>(a, s_plev, s_idp, s_lut, x, y, z, L);
    locate_t<R>(a, h ? t + 0.5 * a.dt : t, L);
    load_cell<F, R>(a, L, c);
    interp_cell<F, R>(a, c, L, out);
  };
  midpoint<R>(a, lon, lat, p, wind, lon, lat, p);
}

// Reflect over the poles, wrap lon to [0, 360), clamp p.  Equal to
// fmod-based wrapping for every input (the short path is exact for
// -360 < lon < 720).
__device__ __forceinline__ void position(const StepArgs &a, double &lon, double &lat, double &p) {
  if (lat > 90.0) {
    lat = 180.0 - lat;
    lon = lon + 180.0;
  } else if (lat < -90.0) {
    lat = -180.0 - lat;
    lon = lon + 180.0;
  }
  double x = lon;
  if (x >= 720.0 || x <= -360.0) x = fmod(x, 360.0);
  else if (x >= 360.0) x = x - 360.0;
  if (x < 0.0) x = x + 360.0;
  if (x >= 360.0) x = 0.0;
  lon = x;
  p = fmin(fmax(p, a.p_top), a.p_bot);
}

// Fickian random walk: sigma_h = sqrt(2 Dx dt), sigma_z = sqrt(2 Dz dt) [m];
// dp = -p dz / H0.
template <typename R>
__device__ __forceinline__ void turb(const StepArgs &a, uint32_t id, uint32_t step, double &lon,
                                     double &lat, double &p) {
  R xi[3];
  normals3<R>(a.seed, id, step, 0u, xi);
  const R kdeg = (R)kDeg;
  const R dx = (R)a.sig_h * xi[0];
  const R dy = (R)a.sig_h * xi[1];
  const R dz = (R)a.sig_z * xi[2];
  const R dlon = dx * kdeg * Math<R>::rcp(cos_floor<R>(a, lat));
  const R dlat = dy * kdeg;
  const R dp = -dz * (R)p * (R)(1.0 / kH0);
  lon = lon + (double)dlon;
  lat = lat + (double)dlat;
  p = p + (double)dp;
}

// turb with the step's normals of purpose 0 (xi) drawn by the caller (the
// same displacement; a copy, so that turb's own code stays as it is).
template <typename R>
__device__ __forceinline__ void turb_drawn(const StepArgs &a, const R xi[3], double &lon, double &lat,
                                           double &p) {
  const R kdeg = (R)kDeg;
  const R dx = (R)a.sig_h * xi[0];
  const R dy = (R)a.sig_h * xi[1];
  const R dz = (R)a.sig_z * xi[2];
  const R dlon = dx * kdeg * Math<R>::rcp(cos_floor<R>(a, lat));
  const R dlat = dy * kdeg;
  const R dp = -dz * (R)p * (R)(1.0 / kH0);
  lon = lon + (double)dlon;
  lat = lat + (double)dlat;
  p = p + (double)dp;
}

// Spread of the 16 values (2 time levels x 2 levels x 2 rows x 2 columns)
// of the cell holding (lon, lat, p) at the time-level pair located by T,
// read from the per-cell table of that pair (one record; k_cell_sigma).
template <typename R>
__device__ __forceinline__ void meso_sigma_table(const StepArgs &a, const double *s_plev,
                                                 const double *s_idp, const uint16_t *s_lut, const TimeLoc &T,
                                                 double lon, double lat, double p, R sg[3]) {
  Loc<R> L;
  locate_xyz<R>(a, s_plev, s_idp, s_lut, lon, lat, p, L);
  set_time(T, L);
  const int off = (L.k * a.ny + L.j) * a.nx + L.i0;            // < 2^31: nx*ny*nz is
  if constexpr (sizeof(R) == 8) {
    const double2 *t = reinterpret_cast<const double2 *>(a.sig) + (size_t)L.l * (size_t)a.level_elems * 2;
    const double2 x = t[2 * off], y = t[2 * off + 1];
    sg[0] = x.x; sg[1] = x.y; sg[2] = y.x;
  } else {
    const float4 *t = reinterpret_cast<const float4 *>(a.sig) + (size_t)L.l * (size_t)a.level_elems;
    const float4 x = t[off];
    sg[0] = x.x; sg[1] = x.y; sg[2] = x.z;
  }
}

// AR(1) update of the sub-grid wind with spread sg, then displacement.
template <typename R>
__device__ __forceinline__ void meso_apply(const StepArgs &a, const R sg[3], const R xi[3],
                                           double &lon, double &lat, double &p, R &up, R &vp, R &wp) {
  const R r = (R)a.r_ar;
  up = fma(r, up, (R)a.rs_fh * sg[0] * xi[0]);
  vp = fma(r, vp, (R)a.rs_fh * sg[1] * xi[1]);
  wp = fma(r, wp, (R)a.rs_fv * sg[2] * xi[2]);
  const R fdt = (R)a.dt;
  const R kdeg = (R)kDeg;
  const R dlon = up * fdt * kdeg * Math<R>::rcp(cos_floor<R>(a, lat));
  const R dlat = vp * fdt * kdeg;
  const R dp = wp * fdt;
  lon = lon + (double)dlon;
  lat = lat + (double)dlat;
  p = p + (double)dp;
}

// AR(1) sub-grid wind from the spread of the 16 values of the current cell
// at the time-level pair of the step's midpoint time (T_mid, from the
// per-cell table), then displacement.
template <int F, typename R>
__device__ __forceinline__ void meso(const StepArgs &a, const double *s_plev, const double *s_idp,
                                     const uint16_t *s_lut, uint32_t id, uint32_t step, const TimeLoc &T_mid,
                                     double &lon, double &lat, double &p, R &up, R &vp, R &wp) {
  R sg[3];
  meso_sigma_table<R>(a, s_plev, s_idp, s_lut, T_mid, lon, lat, p, sg);
  R xi[3];
  normals3<R>(a.seed, id, step, 1u, xi);
  meso_apply<R>(a, sg, xi, lon, lat, p, up, vp, wp);
}

// meso with the step's normals of purpose 1 (xi) drawn by the caller.
template <int F, typename R>
__device__ __forceinline__ void meso_drawn(const StepArgs &a, const double *s_plev, const double *s_idp,
                                           const uint16_t *s_lut, const R xi[3], const TimeLoc &T_mid,
                                           double &lon, double &lat, double &p, R &up, R &vp, R &wp) {
  R sg[3];
  meso_sigma_table<R>(a, s_plev, s_idp, s_lut, T_mid, lon, lat, p, sg);
  meso_apply<R>(a, sg, xi, lon, lat, p, up, vp, wp);
}

// ---- convection and sedimentation ---------------------------------------------

// Temperature at the parcel: the fourth value of the 16 records of its cell
// (R16 storage: decoded with the temperature scale of the (slot, level)),
// time weight first, then lon, lat and p as in interp_cell.  Only that value
// is loaded from each record.
template <int F, typename R>
__device__ __forceinline__ R interp_temp(const StepArgs &a, const Loc<R> &L) {
  using T = typename Rec<F>::T;
  const T *base = reinterpret_cast<const T *>(a.met);
  const int nxy = a.nx * a.ny;
  const int r0 = L.k * nxy + L.j * a.nx;
  using V = typename std::conditional<F == kF32, float, unsigned short>::type;
  V raw[2][2][2][2];                  // [dl][dk][dj][di], all loads issued first
  float sc[2][2];
#pragma unroll
  for (int dl = 0; dl < 2; ++dl) {
    const int slot = dl ? L.l1 : L.l;
#pragma unroll
    for (int dk = 0; dk < 2; ++dk) {
      sc[dl][dk] = F == kF32 ? 1.0f : a.t_scales[slot * a.nz + L.k + dk];
#pragma unroll
      for (int dj = 0; dj < 2; ++dj)
#pragma unroll
        for (int di = 0; di < 2; ++di) {
          const T *rec = base + (int64_t)slot * a.level_elems + r0 + dk * nxy + dj * a.nx + (di ? L.i1 : L.i0);
          raw[dl][dk][dj][di] = reinterpret_cast<const V *>(rec)[3];
        }
    }
  }
  __builtin_amdgcn_s_setprio(0);      // the callers raise it before the locate
  R cv[2][2][2];
#pragma unroll
  for (int dk = 0; dk < 2; ++dk)
#pragma unroll
    for (int dj = 0; dj < 2; ++dj)
#pragma unroll
      for (int di = 0; di < 2; ++di) {
        R v[2];
#pragma unroll
        for (int dl = 0; dl < 2; ++dl) {
          if constexpr (F == kF32) v[dl] = (R)raw[dl][dk][dj][di];
          else v[dl] = (R)(dec<F>(raw[dl][dk][dj][di]) * sc[dl][dk]);
        }
        cv[dk][dj][di] = lerp(v[0], v[1], L.ft);
      }
  R yk[2];
#pragma unroll
  for (int dk = 0; dk < 2; ++dk) {
    const R x0 = lerp(cv[dk][0][0], cv[dk][0][1], L.fx);
    const R x1 = lerp(cv[dk][1][0], cv[dk][1][1], L.fx);
    yk[dk] = lerp(x0, x1, L.fy);
  }
  return lerp(yk[0], yk[1], L.fz);
}

// CAPE, equilibrium-level and surface pressure at the parcel: bilinear in
// (lon, lat) after the time weight at each of the 4 columns.
template <typename R>
__device__ __forceinline__ void interp_sfc(const StepArgs &a, const Loc<R> &L, R out[3]) {
  const int64_t nxy = (int64_t)a.nx * a.ny;
  float4 r0[2][2], r1[2][2];          // all loads issued first
#pragma unroll
  for (int dj = 0; dj < 2; ++dj)
#pragma unroll
    for (int di = 0; di < 2; ++di) {
      const int64_t q = (int64_t)(L.j + dj) * a.nx + (di ? L.i1 : L.i0);
      r0[dj][di] = a.sfc[(int64_t)L.l * nxy + q];
      r1[dj][di] = a.sfc[(int64_t)L.l1 * nxy + q];
    }
  __builtin_amdgcn_s_setprio(0);      // the callers raise it before the locate
  R cv[2][2][3];
#pragma unroll
  for (int dj = 0; dj < 2; ++dj)
#pragma unroll
    for (int di = 0; di < 2; ++di) {
      cv[dj][di][0] = lerp((R)r0[dj][di].x, (R)r1[dj][di].x, L.ft);
      cv[dj][di][1] = lerp((R)r0[dj][di].y, (R)r1[dj][di].y, L.ft);
      cv[dj][di][2] = lerp((R)r0[dj][di].z, (R)r1[dj][di].z, L.ft);
    }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const R x0 = lerp(cv[0][0][q], cv[0][1][q], L.fx);
    const R x1 = lerp(cv[1][0][q], cv[1][1][q], L.fx);
    out[q] = lerp(x0, x1, L.fy);
  }
}

// Unresolved convection: where the CAPE at the parcel reaches the threshold
// and the parcel is below the equilibrium level, it moves to a pressure
// drawn uniformly between the surface and the equilibrium level (equal
// pressure intervals hold equal mass: the column is mixed by mass).  The
// uniform is the first word of the Philox block (id, step, 5, 0), taken in
// FP64 as the new pressure is.
template <int F, typename R>
__device__ __forceinline__ void convection(const StepArgs &a, const double *s_plev,
                                           const double *s_idp, const uint16_t *s_lut, uint32_t id,
                                           uint32_t step, double t_mid, double lon, double lat,
                                           double &p) {
  Loc<R> L;
  __builtin_amdgcn_s_setprio(2);   // locate and gather at raised priority
  locate_xyz<R>(a, s_plev, s_idp, s_lut, lon, lat, p, L);
  locate_t<R>(a, t_mid, L);
  R f[3];
  interp_sfc<R>(a, L, f);
  if (!(f[0] >= (R)a.conv_cape) || !(p > (double)f[1])) return;
  uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  asm("" : "+s"(k0), "+s"(k1) : "s"(step));     // round keys formed per draw, as in normals3
  uint32_t x[4];
  philox4x32_10(id, step, 5u, 0u, k0, k1, x);
  const double ps = (double)f[2], pel = (double)f[1];
  p = ps + (pel - ps) * Math<double>::uni(x[0]);
}

// Sedimentation: settling velocity of a sphere of radius r and density
// rho_p at the parcel's pressure and interpolated temperature (Stokes drag
// with the Cunningham slip correction; Sutherland viscosity; mean free path
// from the mean molecular speed), the parcel sinking v dt metres:
// dp = p v dt / H0, the scale-height conversion of the turbulent step.
template <int F, typename R>
__device__ __forceinline__ void sedimentation(const StepArgs &a, const double *s_plev,
                                              const double *s_idp, const uint16_t *s_lut,
                                              double t_mid, double lon, double lat, double &p) {
  Loc<R> L;
  __builtin_amdgcn_s_setprio(2);   // locate and gather at raised priority
  locate_xyz<R>(a, s_plev, s_idp, s_lut, lon, lat, p, L);
  locate_t<R>(a, t_mid, L);
  const R T = interp_temp<F, R>(a, L);
  const R pr = (R)p;
  const R r = (R)a.sedi_r;
  const R rho = (R)100 * pr / ((R)kRd * T);
  const R eta = (R)1.458e-6 * T * Math<R>::sqrt_(T) / (T + (R)110.4);
  const R vbar = Math<R>::sqrt_((R)(8.0 * kRd / kPi) * T);
  const R kn = (R)2 * eta / (rho * vbar * r);
  const R cc = (R)1 + kn * ((R)1.257 + (R)0.4 * Math<R>::exp_((R)-1.1 / kn));
  const R v = (R)(2.0 * kG / 9.0) * r * r * ((R)a.sedi_rho - rho) * cc / eta;
  p = p + (double)(pr * v * (R)(a.dt / kH0));
}

__device__ __forceinline__ bool finite3(double a, double b, double c) {
  return isfinite(a) && isfinite(b) && isfinite(c);
}

// ---- sort keys ------------------------------------------------------------------

// Sort key of a cell (i0, j, k): its 8 x 8 x 4 tile (tiles numbered lon
// fastest, then lat, then level) times kSubKeys, plus the cell's sub-tile
// inside the tile: kSubLevels halvings of the tile in lon, lat and level,
// each contributing three bits (level, lat, lon from high to low), coarsest
// first.  Consecutive keys then walk a tile's halves in order, so a run of
// sorted parcels that ends one tile and starts the next covers the last
// sub-tiles of one and the first of the other, not both tiles whole.
constexpr int kSubLevels = 1;
constexpr uint32_t kSubKeys = 1u << (3 * kSubLevels);
__host__ __device__ __forceinline__ uint32_t cell_key(int i0, int j, int k, uint32_t ntx, uint32_t nty) {
  uint32_t s = 0;
#pragma unroll
  for (int l = 0; l < kSubLevels; ++l) {
    const int ib = 2 - l, kb = 1 - l;             // the bit each halving tests
    s = (s << 3) | ((uint32_t)((k >> kb) & 1) << 2) | ((uint32_t)((j >> ib) & 1) << 1) | (uint32_t)((i0 >> ib) & 1);
  }
  return (((uint32_t)(k >> 2) * nty + (uint32_t)(j >> 3)) * ntx + (uint32_t)(i0 >> 3)) * kSubKeys + s;
}

// Sort key of a position (cell_key of the cell locate_xyz finds); non-finite
// positions take the last key.
__device__ __forceinline__ uint32_t tile_key(const StepArgs &a, const SortKeyArgs &sk, const double *s_plev,
                                             const uint16_t *s_lut, double lon, double lat, double p) {
  if (!finite3(lon, lat, p)) return sk.nkeys - 1;
  const double lam = lon - 360.0 * floor((lon - a.lon0) * (1.0 / 360.0));
  int i0 = (int)floor((lam - a.lon0) * a.inv_dlon);
  if (i0 >= a.nx) i0 -= a.nx;
  if (i0 < 0) i0 += a.nx;
  const double phi = fmin(fmax(lat, a.lat0), a.lat_hi);
  int j = (int)floor((phi - a.lat0) * a.inv_dlat);
  j = min(max(j, 0), a.ny - 2);
  const int k = level_index(a, s_plev, s_lut, fmin(fmax(p, a.p_top), a.p_bot));
  return cell_key(i0, j, k, sk.ntx, sk.nty);
}

// Rank of each valid lane's key among the parcels of that key: runs of
// equal keys over consecutive valid lanes (invalid lanes may sit anywhere)
// add their length to the key's counter once; a lane's rank is the run's
// old counter value plus its place in the run.  Every lane must call it.
__device__ __forceinline__ uint32_t wave_key_rank(const SortKeyArgs &sk, uint32_t key, bool valid) {
  const int lane = (int)__lane_id();
  const uint32_t prev = __shfl_up(key, 1);
  const uint64_t valids = __ballot(valid);
  const bool prev_valid = lane > 0 && ((valids >> (lane - 1)) & 1ull);
  const uint64_t heads = __ballot(valid && (!prev_valid || prev != key));
  const uint64_t breaks = heads | ~valids;               // a run ends before these lanes
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);   // lanes <= lane
  uint32_t base = 0;
  if ((heads >> lane) & 1ull) {
    const uint64_t above = breaks & ~upto;
    const int end = above ? __ffsll((long long)above) - 1 : 64;
    base = atomicAdd(sk.spread + (key & 15u) * sk.spread_s + (key >> 4), (uint32_t)(end - lane));
  }
  const uint64_t le = heads & upto;
  const int h = le ? 63 - __clzll((long long)le) : 0;
  const uint32_t hb = __shfl(base, h);                  // every lane active
  return hb + (uint32_t)(lane - h);
}

}  // namespace mpt
