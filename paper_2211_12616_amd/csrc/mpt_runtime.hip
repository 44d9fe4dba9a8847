// mpt_runtime.hip -- host side of libmpt: argument validation, workspace
// carving, launch configuration, sort cadence.  Implements include/mpt.h.
#include <math.h>
#include <string.h>

#include <mutex>
#include <new>

#include "../../include/mpt.h"
#include "mpt_internal.h"

using namespace mpt;

struct mpt_ctx {
  mpt_grid grid;
  mpt_params params;
  int device;
  int64_t n_max;
  // workspace carve-out (device)
  unsigned char *ws;
  size_t ws_bytes;
  void *met;              // nt levels
  size_t level_bytes;     // bytes per packed level
  void *sig;              // [nt][npts] spread records of the level pair starting in each slot
  size_t sig_rec;         // 32 (FP64 arithmetic) or 16 bytes; 0 without mesoscale diffusion
  int64_t npts;
  float *scales;          // [nt][3][nz]
  float *t_scales;        // [nt][nz] temperature scales (R16 storage)
  float4 *sfc;            // [nt][ny*nx] {cape, pel, ps, 0}
  double *plev, *inv_dp;  // [nz]
  uint16_t *lut;          // [kLutBins] level lookup table
  float lut_lo, lut_scale;
  int32_t *release;       // [kMaxScen] release step per scenario
  int32_t *rank;          // [kMaxScen] rank of the scenario in release order
  int32_t *rel_sorted;    // [kMaxScen] release steps in ascending order
  uint32_t *step_dev;     // step index read by graph-replayed kernels
  uint32_t *keys, *ranks, *hist, *spread, *block_sums;
  unsigned char *static_scratch;  // this device's copy of the allocation-free sort's scratch
  SortKeyArgs *sk;        // the same buffers for step launches that leave sort keys
  uint32_t ntx, nty, ntz, ntiles, nkeys;
  // host state
  double plev_h[kMaxLevels];
  uint64_t levels_ready;  // bit l set once level l was stored (nt <= 64)
  uint64_t phys_ready;    // bit l set once slot l has its convection / sedimentation fields
  // keys of a step's final positions carried to the next sort (presort):
  // valid for the parcels whose primary lon array and count these are
  bool keyed;
  const double *keyed_lon;
  int64_t keyed_n;
  // a deferred sort's order (in fb_list) for the parcels whose primary lon
  // array and count these are, consumed by the next mpt_step on them
  bool ordered;
  const double *ordered_lon;
  int64_t ordered_n;
  int32_t nscen;
  // surrogate: bf16 weight copies, normalization, training scratch
  uint16_t *s_wt, *s_wb, *s_wi;
  // resident met levels: absolute index of the oldest, its ring slot
  int32_t lev_first, slot_first;
  // gridded output: grid (edges on the device) and whether it is set
  mpt_outgrid og;
  double *out_pe;
  int out_set;
  // hybrid model levels: a[0 .. nml) then b[0 .. nml) on the device
  double *hyb_ab;
  int hyb_nml;
  float *s_norm, *s_bias;               // loaded normalization and biases (FP32)
  uint16_t *s_x;                        // stencil rows of one chunk (bf16 [12][s_chunk][8], chunk-major)
  float *s_y;                           // predictions of one chunk ([s_chunk][4])
  int64_t s_chunk;
  float4 *s_f;                          // FP32 field at a surrogate block's start time
  uint64_t *fb_mask;                    // per wave of 64 parcels: ballot of surrogate fallbacks
  uint32_t *fb_list;                    // indices of the parcels that fall back (n_max)
  uint32_t *fb_off, *fb_sums;           // its prefix sums (+ total) and scan scratch
  float s_tau;
  int s_loaded;
  uint16_t *t_xn, *t_h1, *t_h2, *t_h3, *t_dy, *t_dh1, *t_dh2, *t_dh3;
  float *t_yp, *t_grad, *t_loss_unused;
  double *t_part;
  // captured step loop (mpt_step_graph)
  hipGraph_t graph;
  hipGraphExec_t graph_exec;
  mpt_particles graph_key;
  int32_t graph_nsteps;
};

namespace {

constexpr int kMaxScen = 65536;
constexpr int kMaxTimeLevels = 64;
constexpr int kPersistentBlocks = 2048;   // 256 CUs x 8 blocks

// Scratch of the allocation-free sort (mpt_sort_particles_noalloc): keys
// and ranks of up to MPT_NOALLOC_SORT_MAX_N parcels, the histogram, its
// spread counters and the scan's chunk sums for up to
// MPT_NOALLOC_SORT_MAX_KEYS keys.  One copy per device, held until the
// process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kNaKeys = 0;
constexpr size_t kNaRanks = kNaKeys + sizeof(uint32_t) * (size_t)MPT_NOALLOC_SORT_MAX_N;
constexpr size_t kNaHist = kNaRanks + sizeof(uint32_t) * (size_t)MPT_NOALLOC_SORT_MAX_N;
constexpr size_t kNaSpread = kNaHist + sizeof(uint32_t) * (size_t)MPT_NOALLOC_SORT_MAX_KEYS;
constexpr size_t kNaSums = kNaSpread + sizeof(uint32_t) * (size_t)MPT_NOALLOC_SORT_MAX_KEYS;
constexpr size_t kNaBytes = kNaSums + sizeof(uint32_t) * ((size_t)MPT_NOALLOC_SORT_MAX_KEYS / 1024 + 1);
static_assert(MPT_NOALLOC_SORT_MAX_KEYS % 16 == 0, "the spread counters fill 16 rows");

static __device__ __align__(256) unsigned char scratch[kNaBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices];   // per device, set by the first mpt_create on it

// The device address of `scratch` on device dev (current); null when the
// lookup fails.
unsigned char *scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();          // leave no sticky error for the caller's next call
      return nullptr;
    }
    g_scratch_ptr[dev] = static_cast<unsigned char *>(ptr);
  }
  return g_scratch_ptr[dev];
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

size_t rec_bytes(int dtype) { return dtype == MPT_DT_F32 ? 16 : 8; }

mpt_status check_grid(const mpt_grid *g) {
  if (!g || !g->plev) return MPT_ERR_ARG;
  if (g->nx < 2 || g->ny < 3 || g->nz < 2 || g->nt < 2) return MPT_ERR_ARG;
  if (g->nz > kMaxLevels || g->nt > kMaxTimeLevels) return MPT_ERR_UNSUPPORTED;
  if ((int64_t)g->nx * g->ny * g->nz >= ((int64_t)1 << 31)) return MPT_ERR_UNSUPPORTED;
  if (g->dtype < MPT_DT_F32 || g->dtype > MPT_DT_F16 || g->reserved != 0) return MPT_ERR_ARG;
  if (!(g->dlon > 0) || fabs(g->nx * g->dlon - 360.0) > 1e-9) return MPT_ERR_ARG;
  if (!(g->dlat > 0) || fabs(g->lat0 + 90.0) > 1e-12 ||
      fabs(g->lat0 + (g->ny - 1) * g->dlat - 90.0) > 1e-9)
    return MPT_ERR_ARG;
  if (!isfinite(g->lon0) || !isfinite(g->t_met0) || !(g->dt_met > 0) || !isfinite(g->dt_met))
    return MPT_ERR_ARG;
  for (int k = 0; k < g->nz; ++k) {
    if (!isfinite(g->plev[k]) || !(g->plev[k] > 0)) return MPT_ERR_ARG;
    if (k > 0 && !(g->plev[k] < g->plev[k - 1])) return MPT_ERR_ARG;
  }
  return MPT_OK;
}

mpt_status check_params(const mpt_params *p, const mpt_grid *g) {
  if (!p) return MPT_ERR_ARG;
  if (!(p->dt > 0) || !isfinite(p->dt) || !isfinite(p->t_start)) return MPT_ERR_ARG;
  if (!(p->turb_dx >= 0) || !(p->turb_dz >= 0) || !(p->meso_fh >= 0) || !(p->meso_fv >= 0))
    return MPT_ERR_ARG;
  if (!isfinite(p->turb_dx) || !isfinite(p->turb_dz) || !isfinite(p->meso_fh) || !isfinite(p->meso_fv))
    return MPT_ERR_ARG;
  if (p->sort_interval < 0 || p->fuse < 1) return MPT_ERR_ARG;
  if (p->math != MPT_MATH_F64 && p->math != MPT_MATH_F32) return MPT_ERR_ARG;
  if (p->flags & ~(uint32_t)(MPT_ADVECT | MPT_TURB | MPT_MESO | MPT_CONV | MPT_SEDI)) return MPT_ERR_ARG;
  if ((p->presort != 0 && p->presort != 1) || p->reserved != 0) return MPT_ERR_ARG;
  if ((p->flags & MPT_CONV) && !isfinite(p->conv_cape)) return MPT_ERR_ARG;
  if ((p->flags & MPT_SEDI) && !(isfinite(p->sedi_radius) && p->sedi_radius > 0.0 &&
                                 isfinite(p->sedi_density) && p->sedi_density > 0.0))
    return MPT_ERR_ARG;
  if (p->math == MPT_MATH_F64 && g->dtype != MPT_DT_F32) return MPT_ERR_UNSUPPORTED;
  if (g->dtype != MPT_DT_F32 && r16_max_launch(p->dt, g->dt_met) < 1) return MPT_ERR_UNSUPPORTED;
  return MPT_OK;
}

struct Layout {
  size_t met, sig, scales, t_scales, sfc, sk, plev, inv_dp, lut, release, rank, rel_sorted, step_dev, keys, ranks, hist, spread,
      block_sums, out_pe, hyb_ab, s_wt, s_wb, s_wi, s_norm, s_bias, s_x, s_y, s_f, fb_mask, fb_list, fb_off, fb_sums, t_xn, t_h, t_dy, t_dh, t_yp, t_grad, t_part, total;
  uint32_t ntx, nty, ntz, ntiles, nkeys;
  int64_t s_chunk;
};

// Rows per pass of the surrogate's stencil / MLP / apply kernels.
int64_t surr_chunk(int64_t n_max) {
  int64_t c = n_max > kSurrMaxBatch ? n_max : kSurrMaxBatch;
  c = (c + 63) / 64 * 64;
  return c < kSurrChunk ? c : kSurrChunk;
}

// Bytes per spread record: {su, sv, sw, 0} as double or float; none
// without mesoscale diffusion.
size_t sig_rec_bytes(const mpt_params *p) {
  if (!(p->flags & MPT_MESO)) return 0;
  return p->math == MPT_MATH_F64 ? 32 : 16;
}

Layout layout(const mpt_grid *g, const mpt_params *p, int64_t n_max) {
  Layout L;
  const size_t npts = (size_t)g->nx * g->ny * g->nz;
  L.ntx = (uint32_t)((g->nx + 7) / 8);
  L.nty = (uint32_t)((g->ny - 1 + 7) / 8);
  L.ntz = (uint32_t)((g->nz - 1 + 3) / 4);
  L.ntiles = L.ntx * L.nty * L.ntz * kSubKeys;   // cell keys: tiles x sub-tiles
  L.nkeys = L.ntiles + kMaxScen + 1;
  size_t off = 0;
  L.met = off;        off += align_up(npts * rec_bytes(g->dtype) * g->nt);
  L.sig = off;        off += align_up(npts * sig_rec_bytes(p) * g->nt);
  L.scales = off;     off += align_up(sizeof(float) * 3 * g->nz * g->nt);
  L.t_scales = off;   off += align_up(sizeof(float) * g->nz * g->nt);
  L.sfc = off;        off += align_up((size_t)16 * g->nx * g->ny * g->nt);
  L.sk = off;         off += align_up(sizeof(SortKeyArgs));
  L.plev = off;       off += align_up(sizeof(double) * g->nz);
  L.inv_dp = off;     off += align_up(sizeof(double) * g->nz);
  L.lut = off;        off += align_up(sizeof(uint16_t) * kLutBins);
  L.release = off;    off += align_up(sizeof(int32_t) * kMaxScen);
  L.rank = off;       off += align_up(sizeof(int32_t) * kMaxScen);
  L.rel_sorted = off; off += align_up(sizeof(int32_t) * kMaxScen);
  L.step_dev = off;   off += align_up(sizeof(uint32_t) * 2);
  L.keys = off;       off += align_up(sizeof(uint32_t) * (size_t)(n_max > 0 ? n_max : 0));
  L.ranks = off;      off += align_up(sizeof(uint32_t) * (size_t)(n_max > 0 ? n_max : 0));
  L.hist = off;       off += align_up(sizeof(uint32_t) * L.nkeys);
  L.spread = off;     off += align_up(sizeof(uint32_t) * 16 * ((L.nkeys + 15) / 16));
  L.block_sums = off; off += align_up(sizeof(uint32_t) * scan_block_sums_len(L.nkeys));
  L.out_pe = off;     off += align_up(sizeof(double) * (MPT_MAX_OUT_LEVELS + 1));
  L.hyb_ab = off;     off += align_up(sizeof(double) * 2 * MPT_MAX_ML_LEVELS);
  L.s_wt = off;       off += align_up(sizeof(uint16_t) * kWtSize);
  L.s_wb = off;       off += align_up(sizeof(uint16_t) * kWbSize);
  L.s_wi = off;       off += align_up(sizeof(uint16_t) * kWiSize);
  L.s_norm = off;     off += align_up(sizeof(float) * 12);
  L.s_bias = off;     off += align_up(sizeof(float) * 400);
  L.s_chunk = surr_chunk(n_max);
  L.s_x = off;        off += align_up(sizeof(uint16_t) * (size_t)L.s_chunk * kSurrInPad);
  L.s_y = off;        off += align_up(sizeof(float) * (size_t)L.s_chunk * 4);
  L.s_f = off;        off += g->dtype == MPT_DT_F32 ? align_up(npts * 16) : 0;   // surrogate needs F32 fields
  const size_t nw = (size_t)((n_max > 0 ? n_max : 0) + 63) / 64;
  L.fb_mask = off;    off += align_up(sizeof(uint64_t) * nw);
  L.fb_list = off;    off += align_up(sizeof(uint32_t) * (size_t)(n_max > 0 ? n_max : 0));
  L.fb_off = off;     off += align_up(sizeof(uint32_t) * (nw + 1));
  L.fb_sums = off;    off += align_up(sizeof(uint32_t) * scan_block_sums_len((uint32_t)(nw + 1)));
  L.t_xn = off;       off += align_up(sizeof(uint16_t) * kSurrMaxBatch * kSurrInPad);
  L.t_h = off;        off += align_up(sizeof(uint16_t) * kSurrMaxBatch * kSurrHid * 3);
  L.t_dy = off;       off += align_up(sizeof(uint16_t) * kSurrMaxBatch * kSurrOutPad);
  L.t_dh = off;       off += align_up(sizeof(uint16_t) * kSurrMaxBatch * kSurrHid * 3);
  L.t_yp = off;       off += align_up(sizeof(float) * kSurrMaxBatch * kSurrOutPad);
  L.t_grad = off;     off += align_up(sizeof(float) * kSurrNParam);
  L.t_part = off;     off += align_up(sizeof(double) * kSurrStatBlocks * 84 * 2);
  L.total = off;
  return L;
}

mpt_status from_hip(hipError_t e) { return e == hipSuccess ? MPT_OK : MPT_ERR_HIP; }

void fill_step_args(const mpt_ctx *c, const mpt_particles *P, uint32_t step0, int nsteps,
                    uint32_t flags, StepArgs &a) {
  const mpt_grid &g = c->grid;
  const mpt_params &q = c->params;
  a.lon = P->lon; a.lat = P->lat; a.p = P->p; a.id = P->id;
  a.up = P->up; a.vp = P->vp; a.wp = P->wp;
  a.scen = P->scen;
  a.lev_first = c->lev_first;
  a.slot_first = c->slot_first;
  a.release = P->scen ? c->release : nullptr;
  a.n = P->n;
  a.met = c->met;
  a.level_elems = c->npts;
  a.sig = c->sig;
  a.scales = c->scales;
  a.plev = c->plev;
  a.inv_dp = c->inv_dp;
  a.lut = c->lut;
  a.lut_lo = c->lut_lo;
  a.lut_scale = c->lut_scale;
  a.nx = g.nx; a.ny = g.ny; a.nz = g.nz; a.nt = g.nt;
  a.lon0 = g.lon0; a.inv_dlon = 1.0 / g.dlon;
  a.lat0 = g.lat0; a.inv_dlat = 1.0 / g.dlat;
  a.lat_hi = g.lat0 + (g.ny - 1) * g.dlat;
  a.p_top = c->plev_h[g.nz - 1];
  a.p_bot = c->plev_h[0];
  a.t_met0 = g.t_met0; a.dt_met = g.dt_met; a.inv_dt_met = 1.0 / g.dt_met;
  a.dt = q.dt; a.t_start = q.t_start;
  a.sig_h = sqrt(2.0 * q.turb_dx * q.dt);
  a.sig_z = sqrt(2.0 * q.turb_dz * q.dt);
  double r = 1.0 - 2.0 * q.dt / g.dt_met;
  if (r < 0.0) r = 0.0;
  const double rs = sqrt(1.0 - r * r);
  a.r_ar = r;
  a.rs_fh = rs * q.meso_fh;
  a.rs_fv = rs * q.meso_fv;
  a.cos_cap = cos(89.999 * kPi / 180.0);
  a.seed = q.seed;
  a.step0 = step0;
  a.nsteps = nsteps;
  a.flags = flags;
  const int64_t nblk = (P->n + kBlock - 1) / kBlock;
  a.nblk = (int32_t)nblk;
  a.per_xcd = (int32_t)((nblk + kXcds - 1) / kXcds);
  a.step_dev = nullptr;
  a.persistent = 0;
  a.nscen = c->nscen;
  a.ntiles = c->ntiles;
  a.offsets = c->hist;
  a.rel_sorted = c->rel_sorted;
  a.index = nullptr;
  a.index_count = nullptr;
  a.sk = nullptr;
  a.src = nullptr;
  a.lon_o = a.lat_o = a.p_o = nullptr;
  a.id_o = nullptr;
  a.up_o = a.vp_o = a.wp_o = nullptr;
  a.sfc = c->sfc;
  a.t_scales = c->t_scales;
  a.conv_cape = q.conv_cape;
  a.sedi_r = q.sedi_radius;
  a.sedi_rho = q.sedi_density;
}

mpt_status check_particles(const mpt_ctx *c, const mpt_particles *P, bool need_pingpong,
                           bool need_n_max = true) {
  if (!P) return MPT_ERR_ARG;
  if (P->n < 0) return MPT_ERR_ARG;
  if (P->n > ((int64_t)1 << 31) * kBlock / 2) return MPT_ERR_UNSUPPORTED;
  if (P->n == 0) return MPT_OK;
  const size_t ms = c->params.math == MPT_MATH_F64 ? 8 : 4;
  const bool meso = (c->params.flags & MPT_MESO) != 0;
  if (!P->lon || !P->lat || !P->p || !P->id) return MPT_ERR_ARG;
  if (!aligned(P->lon, 8) || !aligned(P->lat, 8) || !aligned(P->p, 8) || !aligned(P->id, 4))
    return MPT_ERR_ARG;
  if (meso || need_pingpong) {
    if (!P->up || !P->vp || !P->wp) return MPT_ERR_ARG;
    if (!aligned(P->up, ms) || !aligned(P->vp, ms) || !aligned(P->wp, ms)) return MPT_ERR_ARG;
  }
  if (P->scen) {
    if (!aligned(P->scen, 2)) return MPT_ERR_ARG;
    if (c->nscen <= 0) return MPT_ERR_STATE;
  }
  if (need_pingpong) {
    if (need_n_max && P->n > c->n_max) return MPT_ERR_WORKSPACE;
    if (!P->lon2 || !P->lat2 || !P->p2 || !P->id2 || !P->up2 || !P->vp2 || !P->wp2)
      return MPT_ERR_ARG;
    if (!aligned(P->lon2, 8) || !aligned(P->lat2, 8) || !aligned(P->p2, 8) || !aligned(P->id2, 4) ||
        !aligned(P->up2, ms) || !aligned(P->vp2, ms) || !aligned(P->wp2, ms))
      return MPT_ERR_ARG;
    if (P->scen && (!P->scen2 || !aligned(P->scen2, 2))) return MPT_ERR_ARG;
    if (P->lon2 == P->lon || P->id2 == P->id) return MPT_ERR_ARG;
  }
  return MPT_OK;
}

// Every step in [step0, step0 + nsteps) must lie inside the resident levels.
mpt_status check_time(const mpt_ctx *c, uint32_t step0, int64_t nsteps) {
  if (nsteps < 0) return MPT_ERR_ARG;
  if (nsteps == 0) return MPT_OK;
  if ((uint64_t)step0 + (uint64_t)nsteps - 1 > 0xFFFFFFFFull) return MPT_ERR_ARG;
  const mpt_grid &g = c->grid;
  const double t_lo = g.t_met0 + (double)c->lev_first * g.dt_met;
  const double t_hi = g.t_met0 + (double)(c->lev_first + g.nt - 1) * g.dt_met;
  const double eps = 1e-9 * g.dt_met;
  const double t_first = c->params.t_start + (double)step0 * c->params.dt;
  const double t_last_end = c->params.t_start + (double)(step0 + (uint64_t)nsteps - 1) * c->params.dt +
                            c->params.dt;
  if (t_first < t_lo - eps || t_last_end > t_hi + eps) return MPT_ERR_TIME;
  const uint64_t all = (g.nt >= 64) ? ~0ull : ((1ull << g.nt) - 1ull);
  if ((c->levels_ready & all) != all) return MPT_ERR_STATE;
  return MPT_OK;
}

// Sort before step `step` (added to the device step index when dev_step).
// keys_done: the launch before it left the keys of the parcels' current
// positions (and their counts) in the context's sort buffers.
// Scratch of one sort: keys and ranks per parcel, histogram in key order,
// its spread counters, scan chunk sums.
struct SortBufs {
  uint32_t *keys, *ranks, *hist, *spread, *block_sums;
};

void swap_sets(mpt_particles *P);

// inverse: not null = leave the sorted order in inverse (inverse[position] =
// parcel index) instead of moving the state (no swap); the next step launch
// moves it (run_steps with src).
mpt_status do_sort(mpt_ctx *c, mpt_particles *P, uint32_t step, bool dev_step, hipStream_t s,
                   bool keys_done = false, const SortBufs *bufs = nullptr, uint32_t *inverse = nullptr) {
  const SortBufs b = bufs ? *bufs : SortBufs{c->keys, c->ranks, c->hist, c->spread, c->block_sums};
  const mpt_grid &g = c->grid;
  SortArgs sa;
  sa.lon = P->lon; sa.lat = P->lat; sa.p = P->p;
  sa.plev = c->plev; sa.inv_dp = c->inv_dp;
  sa.lut = c->lut; sa.lut_lo = c->lut_lo; sa.lut_scale = c->lut_scale;
  sa.nx = g.nx; sa.ny = g.ny; sa.nz = g.nz;
  sa.lon0 = g.lon0; sa.inv_dlon = 1.0 / g.dlon;
  sa.lat0 = g.lat0; sa.inv_dlat = 1.0 / g.dlat;
  sa.lat_hi = g.lat0 + (g.ny - 1) * g.dlat;
  sa.p_top = c->plev_h[g.nz - 1]; sa.p_bot = c->plev_h[0];
  sa.ntx = c->ntx; sa.nty = c->nty; sa.ntz = c->ntz; sa.nkeys = c->nkeys;
  sa.n = P->n;
  sa.scen = P->scen;
  sa.release = c->release;
  sa.rank = c->rank;
  sa.step = step;
  sa.step_dev = dev_step ? c->step_dev : nullptr;
  sa.keys = b.keys; sa.ranks = b.ranks; sa.hist = b.hist; sa.block_sums = b.block_sums;
  sa.spread = b.spread; sa.spread_s = (c->nkeys + 15) / 16;
  const int64_t nblk = (P->n + kBlock * kSortPer - 1) / (kBlock * kSortPer);
  sa.nblk = (int)nblk;
  sa.per_xcd = (int)((nblk + kXcds - 1) / kXcds);
  ScatterArgs xa;
  xa.n = P->n; xa.keys = b.keys; xa.ranks = b.ranks; xa.offsets = b.hist;
  xa.lon = P->lon; xa.lat = P->lat; xa.p = P->p; xa.id = P->id;
  xa.up = P->up; xa.vp = P->vp; xa.wp = P->wp; xa.scen = P->scen;
  xa.lon2 = P->lon2; xa.lat2 = P->lat2; xa.p2 = P->p2; xa.id2 = P->id2;
  xa.up2 = P->up2; xa.vp2 = P->vp2; xa.wp2 = P->wp2; xa.scen2 = P->scen2;
  xa.meso_bytes = c->params.math == MPT_MATH_F64 ? 8 : 4;
  xa.src = inverse;
  const int64_t nblk_x = (P->n + kBlock - 1) / kBlock;
  xa.nblk = (int)nblk_x;
  xa.per_xcd = (int)((nblk_x + kXcds - 1) / kXcds);
  const mpt_status st = from_hip(launch_sort(sa, xa, keys_done, s));
  if (st != MPT_OK) return st;
  if (!inverse) swap_sets(P);
  return MPT_OK;
}

// The sorted state lives in the *2 set: swap the sets.
void swap_sets(mpt_particles *P) {
  double *t;
  t = P->lon; P->lon = P->lon2; P->lon2 = t;
  t = P->lat; P->lat = P->lat2; P->lat2 = t;
  t = P->p; P->p = P->p2; P->p2 = t;
  uint32_t *ti = P->id; P->id = P->id2; P->id2 = ti;
  void *tv;
  tv = P->up; P->up = P->up2; P->up2 = tv;
  tv = P->vp; P->vp = P->vp2; P->vp2 = tv;
  tv = P->wp; P->wp = P->wp2; P->wp2 = tv;
  uint16_t *ts = P->scen; P->scen = P->scen2; P->scen2 = ts;
}

// persistent: parcels are in the order the last sort of this call left
// them (scenario runs only), so the launch may walk the active prefix.
// keys: the (block-shaped) launch also leaves the sort keys of the final
// positions for the sort that follows.
// src: not null = the deferred sort's order; the launch reads the parcels
// through it and writes the whole state into the *2 set (the caller swaps).
mpt_status run_steps(mpt_ctx *c, const mpt_particles *P, uint32_t step0, int nsteps, uint32_t flags,
                     bool dev_step, bool persistent, hipStream_t s, bool keys = false,
                     const uint32_t *src = nullptr) {
  StepArgs a;
  fill_step_args(c, P, step0, nsteps, flags, a);
  if (src) {
    a.src = src;
    a.lon_o = P->lon2; a.lat_o = P->lat2; a.p_o = P->p2; a.id_o = P->id2;
    a.up_o = P->up2; a.vp_o = P->vp2; a.wp_o = P->wp2;
  }
  if (dev_step) a.step_dev = c->step_dev;
  if (persistent && P->scen) {
    a.persistent = 1;
    a.nblk = kPersistentBlocks;
  }
  if (keys) {
    if (launch_clear_spread(c->spread, (c->nkeys + 15) / 16, s) != hipSuccess) return MPT_ERR_HIP;
    a.sk = c->sk;
  }
  return from_hip(launch_step(c->grid.dtype, c->params.math == MPT_MATH_F64, a, s));
}

// The launch sequence of steps [first, first + count), all of them inside
// one sort window or starting with its sort: sort at window starts, fused
// launches of at most params.fuse steps.  Step indices are offsets from the
// device step index when dev_step.
// Without scenarios, a launch that ends where a sort follows also leaves
// the sort keys of its final positions, and that sort skips its key pass;
// with params.presort the call's last launch does the same and the keys are
// kept for the next sort of the same parcels (mpt_sort_particles, or the
// sort the next call starts with).  Graph-captured sequences (dev_step)
// keep nothing across calls.
mpt_status enqueue_steps(mpt_ctx *c, mpt_particles *P, int64_t first, int64_t count, bool dev_step,
                         hipStream_t s) {
  const int S = c->params.sort_interval;
  const uint32_t flags = c->params.flags;
  // keys carried from the previous call hold for a sort this call starts with
  bool keys_ready = S > 0 && !P->scen && !dev_step && c->keyed && c->keyed_lon == P->lon &&
                    c->keyed_n == P->n && first % S == 0;
  c->keyed = false;
  bool sorted = false;
  int64_t cur = first;
  const int64_t end = first + count;
  // Without scenarios and outside graph capture, a sort followed by a
  // step launch is deferred into it: the sort leaves its order as a list
  // (in the fallback-list buffer, free outside the surrogate) and the launch
  // reads its parcels through it and writes them in sorted order, so the
  // state moves once instead of twice.
  const bool defer = flags && !P->scen && !dev_step && P->n <= c->n_max;
  // a deferred sort of these parcels (mpt_sort_particles_deferred) is
  // completed by the first launch, unless this call starts with its own sort
  const uint32_t *order =
      defer && c->ordered && c->ordered_lon == P->lon && c->ordered_n == P->n ? c->fb_list : nullptr;
  c->ordered = false;
  while (cur < end) {
    if (S > 0 && cur % S == 0) {
      mpt_status st = do_sort(c, P, (uint32_t)cur, dev_step, s, keys_ready, nullptr, defer ? c->fb_list : nullptr);
      if (st != MPT_OK) return st;
      sorted = true;
      order = defer ? c->fb_list : nullptr;
    }
    keys_ready = false;
    int64_t stop = end;
    if (S > 0) {
      const int64_t next_sort = (cur / S + 1) * S;
      if (next_sort < stop) stop = next_sort;
    }
    if (stop - cur > c->params.fuse) stop = cur + c->params.fuse;
    if (c->grid.dtype != MPT_DT_F32) {
      const int cap = r16_max_launch(c->params.dt, c->grid.dt_met);
      if (stop - cur > cap) stop = cur + cap;
    }
    if (flags) {
      // (the key buffers hold n_max parcels)
      const bool keys = !P->scen && P->n <= c->n_max &&
                        (stop < end ? S > 0 && stop % S == 0 : c->params.presort && !dev_step);
      mpt_status st = run_steps(c, P, (uint32_t)cur, (int)(stop - cur), flags, dev_step, sorted, s, keys, order);
      if (st != MPT_OK) return st;
      if (order) {
        swap_sets(P);
        order = nullptr;
      }
      keys_ready = keys;
    }
    cur = stop;
  }
  if (keys_ready) {
    c->keyed = true;
    c->keyed_lon = P->lon;
    c->keyed_n = P->n;
  }
  return MPT_OK;
}

// Weight views: bf16 copies in the context plus FP32 biases and
// normalization at the given addresses.
SurrW surr_weights(const mpt_ctx *c, const float *params, const float *norm) {
  SurrW W;
  W.wt1 = c->s_wt;
  W.wt2 = W.wt1 + kSurrHid * kSurrInPad;
  W.wt3 = W.wt2 + kSurrHid * kSurrHid;
  W.wt4 = W.wt3 + kSurrHid * kSurrHid;
  W.wb2 = c->s_wb;
  W.wb3 = W.wb2 + kSurrHid * kSurrHid;
  W.wb4 = W.wb3 + kSurrHid * kSurrHid;
  W.b1 = params + kOffB1;
  W.b2 = params + kOffB2;
  W.b3 = params + kOffB3;
  W.b4 = params + kOffB4;
  W.norm = norm;
  W.wi = c->s_wi;
  return W;
}

void drop_graph(mpt_ctx *c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
}

}  // namespace

extern "C" {

size_t mpt_workspace_bytes(const mpt_grid *grid, const mpt_params *params, int64_t n_max) {
  if (check_grid(grid) != MPT_OK || check_params(params, grid) != MPT_OK || n_max < 0) return 0;
  if (n_max >= kMaxParcels) return 0;
  return layout(grid, params, n_max).total;
}

mpt_status mpt_create(const mpt_grid *grid, const mpt_params *params, int64_t n_max,
                      void *dev_workspace, size_t ws_bytes, mpt_ctx **out) {
  if (!out) return MPT_ERR_ARG;
  *out = nullptr;
  mpt_status st = check_grid(grid);
  if (st != MPT_OK) return st;
  st = check_params(params, grid);
  if (st != MPT_OK) return st;
  if (n_max < 0) return MPT_ERR_ARG;
  if (n_max >= kMaxParcels) return MPT_ERR_UNSUPPORTED;
  if (!dev_workspace || !aligned(dev_workspace, 256)) return MPT_ERR_ARG;
  const Layout L = layout(grid, params, n_max);
  if (ws_bytes < L.total) return MPT_ERR_WORKSPACE;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return MPT_ERR_HIP;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MPT_ERR_HIP;

  mpt_ctx *c = new (std::nothrow) mpt_ctx();
  if (!c) return MPT_ERR_HIP;
  c->grid = *grid;
  c->params = *params;
  c->device = dev;
  c->n_max = n_max;
  for (int k = 0; k < grid->nz; ++k) c->plev_h[k] = grid->plev[k];
  c->grid.plev = c->plev_h;
  unsigned char *ws = static_cast<unsigned char *>(dev_workspace);
  c->ws = ws;
  c->ws_bytes = ws_bytes;
  c->npts = (int64_t)grid->nx * grid->ny * grid->nz;
  c->level_bytes = (size_t)c->npts * rec_bytes(grid->dtype);
  c->met = ws + L.met;
  c->sig_rec = sig_rec_bytes(params);
  c->sig = c->sig_rec ? ws + L.sig : nullptr;
  c->scales = reinterpret_cast<float *>(ws + L.scales);
  c->t_scales = reinterpret_cast<float *>(ws + L.t_scales);
  c->sfc = reinterpret_cast<float4 *>(ws + L.sfc);
  c->sk = reinterpret_cast<SortKeyArgs *>(ws + L.sk);
  c->plev = reinterpret_cast<double *>(ws + L.plev);
  c->inv_dp = reinterpret_cast<double *>(ws + L.inv_dp);
  c->lut = reinterpret_cast<uint16_t *>(ws + L.lut);
  c->release = reinterpret_cast<int32_t *>(ws + L.release);
  c->rank = reinterpret_cast<int32_t *>(ws + L.rank);
  c->rel_sorted = reinterpret_cast<int32_t *>(ws + L.rel_sorted);
  c->step_dev = reinterpret_cast<uint32_t *>(ws + L.step_dev);
  c->keys = reinterpret_cast<uint32_t *>(ws + L.keys);
  c->ranks = reinterpret_cast<uint32_t *>(ws + L.ranks);
  c->hist = reinterpret_cast<uint32_t *>(ws + L.hist);
  c->spread = reinterpret_cast<uint32_t *>(ws + L.spread);
  c->block_sums = reinterpret_cast<uint32_t *>(ws + L.block_sums);
  c->static_scratch = scratch_address(dev);
  c->out_pe = reinterpret_cast<double *>(ws + L.out_pe);
  c->hyb_ab = reinterpret_cast<double *>(ws + L.hyb_ab);
  c->ntx = L.ntx; c->nty = L.nty; c->ntz = L.ntz; c->ntiles = L.ntiles; c->nkeys = L.nkeys;
  c->s_wt = reinterpret_cast<uint16_t *>(ws + L.s_wt);
  c->s_wb = reinterpret_cast<uint16_t *>(ws + L.s_wb);
  c->s_wi = reinterpret_cast<uint16_t *>(ws + L.s_wi);
  c->s_norm = reinterpret_cast<float *>(ws + L.s_norm);
  c->s_bias = reinterpret_cast<float *>(ws + L.s_bias);
  c->s_x = reinterpret_cast<uint16_t *>(ws + L.s_x);
  c->s_y = reinterpret_cast<float *>(ws + L.s_y);
  c->s_chunk = L.s_chunk;
  c->s_f = reinterpret_cast<float4 *>(ws + L.s_f);
  c->fb_mask = reinterpret_cast<uint64_t *>(ws + L.fb_mask);
  c->fb_list = reinterpret_cast<uint32_t *>(ws + L.fb_list);
  c->fb_off = reinterpret_cast<uint32_t *>(ws + L.fb_off);
  c->fb_sums = reinterpret_cast<uint32_t *>(ws + L.fb_sums);
  c->t_xn = reinterpret_cast<uint16_t *>(ws + L.t_xn);
  c->t_h1 = reinterpret_cast<uint16_t *>(ws + L.t_h);
  c->t_h2 = c->t_h1 + (size_t)kSurrMaxBatch * kSurrHid;
  c->t_h3 = c->t_h2 + (size_t)kSurrMaxBatch * kSurrHid;
  c->t_dy = reinterpret_cast<uint16_t *>(ws + L.t_dy);
  c->t_dh1 = reinterpret_cast<uint16_t *>(ws + L.t_dh);
  c->t_dh2 = c->t_dh1 + (size_t)kSurrMaxBatch * kSurrHid;
  c->t_dh3 = c->t_dh2 + (size_t)kSurrMaxBatch * kSurrHid;
  c->t_yp = reinterpret_cast<float *>(ws + L.t_yp);
  c->t_grad = reinterpret_cast<float *>(ws + L.t_grad);
  c->t_part = reinterpret_cast<double *>(ws + L.t_part);

  double idp[kMaxLevels];
  for (int k = 0; k < grid->nz - 1; ++k) idp[k] = 1.0 / (grid->plev[k] - grid->plev[k + 1]);
  idp[grid->nz - 1] = 0.0;
  // level lookup table: bin b of log2(p) starts the search at the largest k
  // whose level is at or below the bin's upper pressure edge
  const double lo = log2(grid->plev[grid->nz - 1]), hi = log2(grid->plev[0]);
  const double scale = kLutBins / (hi - lo);
  uint16_t lut[kLutBins];
  int k = grid->nz - 2;
  for (int b = 0; b < kLutBins; ++b) {            // upper edges rise with b, k falls
    const double p_hi = exp2(lo + (b + 1) / scale);
    while (k > 0 && grid->plev[k] < p_hi) --k;
    lut[b] = (uint16_t)k;
  }
  c->lut_lo = (float)lo;
  c->lut_scale = (float)scale;
  SortKeyArgs skh;
  skh.keys = c->keys;
  skh.ranks = c->ranks;
  skh.spread = c->spread;
  skh.spread_s = (c->nkeys + 15) / 16;
  skh.ntx = c->ntx;
  skh.nty = c->nty;
  skh.nkeys = c->nkeys;
  if (hipMemcpy(c->sk, &skh, sizeof(skh), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->plev, c->plev_h, sizeof(double) * grid->nz, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->inv_dp, idp, sizeof(double) * grid->nz, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->lut, lut, sizeof(uint16_t) * kLutBins, hipMemcpyHostToDevice) != hipSuccess) {
    delete c;
    return MPT_ERR_HIP;
  }
  if (launch_fill_f32(c->scales, 1.0f, (int64_t)3 * grid->nz * grid->nt, nullptr) != hipSuccess ||
      hipStreamSynchronize(nullptr) != hipSuccess) {
    delete c;
    return MPT_ERR_HIP;
  }
  *out = c;
  return MPT_OK;
}

namespace {
// Pack a time level from device arrays into ring slot `slot` (F32 records,
// or R16 codes with their per-level scales).
mpt_status pack_level(mpt_ctx *c, int slot, const float *u, const float *v, const float *w,
                      hipStream_t s) {
  const int64_t nxy = (int64_t)c->grid.nx * c->grid.ny;
  unsigned char *dst = static_cast<unsigned char *>(c->met) + c->level_bytes * (size_t)slot;
  float *sc = c->scales + (size_t)slot * 3 * c->grid.nz;
  hipError_t e;
  if (c->grid.dtype == MPT_DT_F32) {
    e = launch_pack_f32(u, v, w, reinterpret_cast<float4 *>(dst), c->npts, s);
  } else {
    e = launch_level_absmax(u, v, w, nxy, c->grid.nz, sc, s);
    if (e == hipSuccess)
      e = launch_pack_r16(c->grid.dtype, u, v, w, sc, reinterpret_cast<ushort4 *>(dst), nxy,
                          c->grid.nz, s);
  }
  if (e != hipSuccess) return MPT_ERR_HIP;
  c->phys_ready &= ~(1ull << slot);     // the records' fourth values were cleared
  return MPT_OK;
}

// Spread tables of the level pairs that include resident level `pos`
// (0 .. nt-1 from the oldest): pairs (pos-1, pos) and (pos, pos+1), when both
// of their levels are stored.  A pair's table sits in the slot of its
// earlier level.
mpt_status update_sigma(mpt_ctx *c, int pos, hipStream_t s) {
  if (!c->sig) return MPT_OK;
  const int nt = c->grid.nt;
  for (int q = pos - 1; q <= pos; ++q) {
    if (q < 0 || q > nt - 2) continue;
    const int s0 = (c->slot_first + q) % nt, s1 = (s0 + 1) % nt;
    if (!(c->levels_ready & (1ull << s0)) || !(c->levels_ready & (1ull << s1))) continue;
    void *out = static_cast<unsigned char *>(c->sig) + c->sig_rec * (size_t)c->npts * (size_t)s0;
    if (launch_cell_sigma(c->grid.dtype, c->sig_rec == 32, c->met, c->scales, s0, s1, c->npts, c->grid.nx,
                          c->grid.ny, c->grid.nz, out, s) != hipSuccess)
      return MPT_ERR_HIP;
  }
  return MPT_OK;
}

// The convection / sedimentation fields must be stored on every resident
// level when the step uses them.
mpt_status check_phys(const mpt_ctx *c) {
  if (!(c->params.flags & (MPT_CONV | MPT_SEDI))) return MPT_OK;
  const uint64_t all = (c->grid.nt >= 64) ? ~0ull : ((1ull << c->grid.nt) - 1ull);
  return (c->phys_ready & all) == all ? MPT_OK : MPT_ERR_STATE;
}
}  // namespace

mpt_status mpt_set_met_phys(mpt_ctx *c, int32_t level, const float *temp, const float *cape,
                            const float *pel, const float *ps, void *hip_stream) {
  if (!c || !temp || !cape || !pel || !ps) return MPT_ERR_ARG;
  if (level < 0 || level >= c->grid.nt) return MPT_ERR_ARG;
  if (!aligned(temp, 4) || !aligned(cape, 4) || !aligned(pel, 4) || !aligned(ps, 4)) return MPT_ERR_ARG;
  const int slot = (c->slot_first + level) % c->grid.nt;
  if (!(c->levels_ready & (1ull << slot))) return MPT_ERR_STATE;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int64_t nxy = (int64_t)c->grid.nx * c->grid.ny;
  void *dst = static_cast<unsigned char *>(c->met) + c->level_bytes * (size_t)slot;
  hipError_t e = launch_pack_temp(c->grid.dtype, temp, c->t_scales + (size_t)slot * c->grid.nz, dst, nxy,
                                  c->grid.nz, s);
  if (e == hipSuccess) e = launch_pack_sfc(cape, pel, ps, c->sfc + (size_t)slot * nxy, nxy, s);
  if (e != hipSuccess) return MPT_ERR_HIP;
  c->phys_ready |= 1ull << slot;
  return MPT_OK;
}

mpt_status mpt_init_met(mpt_ctx *c, int32_t level, const float *u, const float *v, const float *w,
                        void *hip_stream) {
  if (!c || !u || !v || !w) return MPT_ERR_ARG;
  if (level < 0 || level >= c->grid.nt) return MPT_ERR_ARG;
  if (!aligned(u, 4) || !aligned(v, 4) || !aligned(w, 4)) return MPT_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int slot = (c->slot_first + level) % c->grid.nt;
  const mpt_status st = pack_level(c, slot, u, v, w, s);
  if (st != MPT_OK) return st;
  c->levels_ready |= 1ull << slot;
  return update_sigma(c, level, s);
}

mpt_status mpt_push_met(mpt_ctx *c, const float *u, const float *v, const float *w, void *hip_stream) {
  if (!c || !u || !v || !w) return MPT_ERR_ARG;
  if (!aligned(u, 4) || !aligned(v, 4) || !aligned(w, 4)) return MPT_ERR_ARG;
  const uint64_t all = (c->grid.nt >= 64) ? ~0ull : ((1ull << c->grid.nt) - 1ull);
  if ((c->levels_ready & all) != all) return MPT_ERR_STATE;
  if (c->lev_first > 0x7FFFFFFF - c->grid.nt - 1) return MPT_ERR_UNSUPPORTED;
  // the oldest level's slot receives level lev_first + nt
  const mpt_status st = pack_level(c, c->slot_first, u, v, w, static_cast<hipStream_t>(hip_stream));
  if (st != MPT_OK) return st;
  c->lev_first += 1;
  c->slot_first = c->slot_first + 1 == c->grid.nt ? 0 : c->slot_first + 1;
  drop_graph(c);                        // captured launches hold the old window
  return update_sigma(c, c->grid.nt - 1, static_cast<hipStream_t>(hip_stream));
}



size_t mpt_met_level_bytes(const mpt_ctx *c) { return c ? c->level_bytes : 0; }

mpt_status mpt_copy_met_level(mpt_ctx *c, int32_t level, void *dst, float *scales_dst,
                              void *hip_stream) {
  if (!c || !dst || !scales_dst) return MPT_ERR_ARG;
  if (level < 0 || level >= c->grid.nt) return MPT_ERR_ARG;
  level = (c->slot_first + level) % c->grid.nt;          // its ring slot
  if (!(c->levels_ready & (1ull << level))) return MPT_ERR_STATE;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const unsigned char *src = static_cast<const unsigned char *>(c->met) + c->level_bytes * (size_t)level;
  if (hipMemcpyAsync(dst, src, c->level_bytes, hipMemcpyDeviceToDevice, s) != hipSuccess) return MPT_ERR_HIP;
  if (hipMemcpyAsync(scales_dst, c->scales + (size_t)level * 3 * c->grid.nz,
                     sizeof(float) * 3 * c->grid.nz, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return MPT_ERR_HIP;
  return MPT_OK;
}

mpt_status mpt_set_release(mpt_ctx *c, int32_t nscen, const int32_t *release_step, void *hip_stream) {
  if (!c || !release_step || nscen < 1 || nscen > kMaxScen) return MPT_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // rank of each scenario in release order (ties by index), sorted table
  int32_t *order = new (std::nothrow) int32_t[nscen];
  int32_t *rank = new (std::nothrow) int32_t[nscen];
  int32_t *sorted = new (std::nothrow) int32_t[nscen];
  if (!order || !rank || !sorted) {
    delete[] order; delete[] rank; delete[] sorted;
    return MPT_ERR_HIP;
  }
  for (int i = 0; i < nscen; ++i) order[i] = i;
  // insertion sort by (release, index): stable, nscen <= 65536
  for (int i = 1; i < nscen; ++i) {
    const int32_t v = order[i];
    int j = i - 1;
    while (j >= 0 && release_step[order[j]] > release_step[v]) {
      order[j + 1] = order[j];
      --j;
    }
    order[j + 1] = v;
  }
  for (int r = 0; r < nscen; ++r) {
    rank[order[r]] = r;
    sorted[r] = release_step[order[r]];
  }
  // copied synchronously: the host arrays may be reused right after the call
  const bool ok =
      hipMemcpyAsync(c->release, release_step, sizeof(int32_t) * nscen, hipMemcpyHostToDevice, s) ==
          hipSuccess &&
      hipMemcpyAsync(c->rank, rank, sizeof(int32_t) * nscen, hipMemcpyHostToDevice, s) == hipSuccess &&
      hipMemcpyAsync(c->rel_sorted, sorted, sizeof(int32_t) * nscen, hipMemcpyHostToDevice, s) ==
          hipSuccess &&
      hipStreamSynchronize(s) == hipSuccess;
  delete[] order; delete[] rank; delete[] sorted;
  if (!ok) return MPT_ERR_HIP;
  c->nscen = nscen;
  drop_graph(c);
  return MPT_OK;
}

mpt_status mpt_advect(mpt_ctx *c, const mpt_particles *P, uint32_t step, void *hip_stream) {
  if (!c) return MPT_ERR_ARG;
  mpt_status st = check_particles(c, P, false);
  if (st != MPT_OK) return st;
  st = check_time(c, step, 1);
  if (st != MPT_OK) return st;
  c->keyed = false;                                  // positions move
  c->ordered = false;
  if (P->n == 0 || !(c->params.flags & MPT_ADVECT)) return MPT_OK;
  return run_steps(c, P, step, 1, MPT_ADVECT, false, false, static_cast<hipStream_t>(hip_stream));
}

mpt_status mpt_diffuse(mpt_ctx *c, const mpt_particles *P, uint32_t step, void *hip_stream) {
  if (!c) return MPT_ERR_ARG;
  mpt_status st = check_particles(c, P, false);
  if (st != MPT_OK) return st;
  st = check_time(c, step, 1);
  if (st != MPT_OK) return st;
  c->keyed = false;                                  // positions move
  c->ordered = false;
  const uint32_t f = c->params.flags & (MPT_TURB | MPT_MESO);
  if (P->n == 0 || !f) return MPT_OK;
  return run_steps(c, P, step, 1, f, false, false, static_cast<hipStream_t>(hip_stream));
}

mpt_status mpt_sort_particles(mpt_ctx *c, mpt_particles *P, void *hip_stream) {
  if (!c) return MPT_ERR_ARG;
  const mpt_status st = check_particles(c, P, true);
  if (st != MPT_OK) return st;
  if (P->n == 0) return MPT_OK;
  const bool keys_done = c->keyed && !P->scen && c->keyed_lon == P->lon && c->keyed_n == P->n;
  c->keyed = false;
  c->ordered = false;
  return do_sort(c, P, 0u, false, static_cast<hipStream_t>(hip_stream), keys_done);
}

mpt_status mpt_sort_particles_deferred(mpt_ctx *c, mpt_particles *P, void *hip_stream) {
  if (!c) return MPT_ERR_ARG;
  const mpt_status st = check_particles(c, P, true);
  if (st != MPT_OK) return st;
  c->ordered = false;
  if (P->n == 0) return MPT_OK;
  const bool keys_done = c->keyed && !P->scen && c->keyed_lon == P->lon && c->keyed_n == P->n;
  c->keyed = false;
  const mpt_status r = do_sort(c, P, 0u, false, static_cast<hipStream_t>(hip_stream), keys_done, nullptr,
                               c->fb_list);
  if (r != MPT_OK) return r;
  c->ordered = true;
  c->ordered_lon = P->lon;
  c->ordered_n = P->n;
  return MPT_OK;
}

mpt_status mpt_sort_particles_noalloc(mpt_ctx *c, mpt_particles *P, void *hip_stream) {
  if (!c) return MPT_ERR_ARG;
  if (P && P->n > MPT_NOALLOC_SORT_MAX_N) return MPT_ERR_WORKSPACE;
  if (c->nkeys > (uint32_t)MPT_NOALLOC_SORT_MAX_KEYS) return MPT_ERR_UNSUPPORTED;
  const mpt_status st = check_particles(c, P, true, /*need_n_max=*/false);
  if (st != MPT_OK) return st;
  if (P->n == 0) return MPT_OK;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || !c->static_scratch) return MPT_ERR_HIP;
  if (dev != c->device) return MPT_ERR_STATE;     // the scratch address is the context's device's
  c->keyed = false;                    // the keys a step left are not used here
  c->ordered = false;
  unsigned char *base = c->static_scratch;
  const SortBufs b{reinterpret_cast<uint32_t *>(base + kNaKeys), reinterpret_cast<uint32_t *>(base + kNaRanks),
                   reinterpret_cast<uint32_t *>(base + kNaHist), reinterpret_cast<uint32_t *>(base + kNaSpread),
                   reinterpret_cast<uint32_t *>(base + kNaSums)};
  return do_sort(c, P, 0u, false, static_cast<hipStream_t>(hip_stream), false, &b);
}

mpt_status mpt_step(mpt_ctx *c, mpt_particles *P, uint32_t step0, int32_t nsteps, void *hip_stream) {
  if (!c) return MPT_ERR_ARG;
  const int S = c->params.sort_interval;
  bool sorts = false;
  if (S > 0 && nsteps > 0) {
    for (int64_t s = step0; s < (int64_t)step0 + nsteps; ++s)
      if (s % S == 0) { sorts = true; break; }
  }
  mpt_status st = check_particles(c, P, sorts);
  if (st != MPT_OK) return st;
  st = check_time(c, step0, nsteps);
  if (st != MPT_OK) return st;
  st = check_phys(c);
  if (st != MPT_OK) return st;
  if (P->n == 0 || nsteps == 0) return MPT_OK;
  return enqueue_steps(c, P, step0, nsteps, false, static_cast<hipStream_t>(hip_stream));
}

mpt_status mpt_step_graph(mpt_ctx *c, mpt_particles *P, uint32_t step0, int32_t nsteps,
                          void *hip_stream) {
  if (!c) return MPT_ERR_ARG;
  const int S = c->params.sort_interval;
  if (!hip_stream) return MPT_ERR_ARG;                 // capture needs a created stream
  if (S <= 0 || step0 % (uint32_t)S != 0 || nsteps < 0 || nsteps % (2 * S) != 0)
    return MPT_ERR_ARG;
  mpt_status st = check_particles(c, P, nsteps > 0);
  if (st != MPT_OK) return st;
  st = check_time(c, step0, nsteps);
  if (st != MPT_OK) return st;
  st = check_phys(c);
  if (st != MPT_OK) return st;
  if (P->n == 0 || nsteps == 0) return MPT_OK;
  c->keyed = false;                                  // replays keep no keys across calls
  c->ordered = false;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const bool same = c->graph_exec && memcmp(&c->graph_key, P, sizeof(*P)) == 0 &&
                    c->graph_nsteps == 2 * S;
  if (!same) {
    drop_graph(c);
    mpt_particles Q = *P;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return MPT_ERR_HIP;
    st = enqueue_steps(c, &Q, 0, 2 * S, true, s);
    if (st == MPT_OK && launch_add_u32(c->step_dev, (uint32_t)(2 * S), s) != hipSuccess) st = MPT_ERR_HIP;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (st != MPT_OK || e != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return st != MPT_OK ? st : MPT_ERR_HIP;
    }
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      return MPT_ERR_HIP;
    }
    c->graph = g;
    c->graph_exec = x;
    c->graph_key = *P;
    c->graph_nsteps = 2 * S;
  }
  if (launch_set_u32(c->step_dev, step0, s) != hipSuccess) return MPT_ERR_HIP;
  for (int32_t r = 0; r < nsteps / (2 * S); ++r)
    if (hipGraphLaunch(c->graph_exec, s) != hipSuccess) return MPT_ERR_HIP;
  return MPT_OK;
}

// ---- surrogate ------------------------------------------------------------------

mpt_status mpt_surrogate_datagen(mpt_ctx *c, int64_t n, const double *lon, const double *lat,
                                 const double *p, const uint32_t *step, float *x, float *y,
                                 void *hip_stream) {
  if (!c) return MPT_ERR_ARG;
  if (n < 0 || (n > 0 && (!lon || !lat || !p || !step || !x || !y))) return MPT_ERR_ARG;
  if (c->grid.dtype != MPT_DT_F32) return MPT_ERR_UNSUPPORTED;
  const uint64_t all = (c->grid.nt >= 64) ? ~0ull : ((1ull << c->grid.nt) - 1ull);
  if ((c->levels_ready & all) != all) return MPT_ERR_STATE;
  if (n == 0) return MPT_OK;
  mpt_particles P = {};
  P.n = n;
  StepArgs a;
  fill_step_args(c, &P, 0, kSurrK, MPT_ADVECT, a);
  return from_hip(launch_surr_datagen(a, n, lon, lat, p, step, x, y, static_cast<hipStream_t>(hip_stream)));
}

mpt_status mpt_surrogate_stats(mpt_ctx *c, int64_t n, const float *x, const float *y, float *norm,
                               void *hip_stream) {
  if (!c || n < 1 || !x || !y || !norm) return MPT_ERR_ARG;
  const int nblk = (int)(n < kSurrStatBlocks ? n : kSurrStatBlocks);
  return from_hip(launch_surr_stats(x, y, n, c->t_part, nblk, norm, static_cast<hipStream_t>(hip_stream)));
}

mpt_status mpt_surrogate_init(mpt_ctx *c, float *params, uint64_t seed, void *hip_stream) {
  if (!c || !params) return MPT_ERR_ARG;
  return from_hip(launch_surr_init(params, seed, static_cast<hipStream_t>(hip_stream)));
}

mpt_status mpt_surrogate_train_step(mpt_ctx *c, const float *x, const float *y, int32_t batch,
                                    const float *norm, float *params, float *adam_m, float *adam_v,
                                    int32_t t, float lr, float *loss, void *hip_stream) {
  if (!c || !x || !y || !norm || !params || !adam_m || !adam_v || !loss) return MPT_ERR_ARG;
  if (batch < 64 || batch > kSurrMaxBatch || batch % 64 != 0 || t < 1 || !(lr > 0.0f)) return MPT_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // bf16 copies of the current weights, then forward, backward, Adam
  if (launch_surr_pack(params, c->s_wt, c->s_wb, s) != hipSuccess) return MPT_ERR_HIP;
  const SurrW W = surr_weights(c, params, norm);
  SurrTrain T;
  T.x = x; T.y = y; T.batch = batch;
  T.xn = c->t_xn; T.h1 = c->t_h1; T.h2 = c->t_h2; T.h3 = c->t_h3;
  T.dy = c->t_dy; T.dh1 = c->t_dh1; T.dh2 = c->t_dh2; T.dh3 = c->t_dh3;
  T.yp = c->t_yp; T.grad = c->t_grad; T.loss = loss;
  const float bc1 = 1.0f - powf(0.9f, (float)t), bc2 = 1.0f - powf(0.999f, (float)t);
  c->s_loaded = 0;                      // the copies now hold training weights
  return from_hip(launch_surr_train(W, T, params, adam_m, adam_v, lr, bc1, bc2, s));
}

mpt_status mpt_surrogate_grad(mpt_ctx *c, const float *x, const float *y, int32_t batch,
                              const float *norm, const float *params, float *grad, float *loss,
                              void *hip_stream) {
  if (!c || !x || !y || !norm || !params || !grad || !loss) return MPT_ERR_ARG;
  if (batch < 64 || batch > kSurrMaxBatch || batch % 64 != 0) return MPT_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (launch_surr_pack(params, c->s_wt, c->s_wb, s) != hipSuccess) return MPT_ERR_HIP;
  const SurrW W = surr_weights(c, params, norm);
  SurrTrain T;
  T.x = x; T.y = y; T.batch = batch;
  T.xn = c->t_xn; T.h1 = c->t_h1; T.h2 = c->t_h2; T.h3 = c->t_h3;
  T.dy = c->t_dy; T.dh1 = c->t_dh1; T.dh2 = c->t_dh2; T.dh3 = c->t_dh3;
  T.yp = c->t_yp; T.grad = grad; T.loss = loss;
  c->s_loaded = 0;
  return from_hip(launch_surr_grad(W, T, s));
}

mpt_status mpt_surrogate_load(mpt_ctx *c, const float *params, const float *norm, float tau_km,
                              void *hip_stream) {
  if (!c || !params || !norm || !(tau_km >= 0.0f)) return MPT_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (launch_surr_pack(params, c->s_wt, c->s_wb, s) != hipSuccess ||
      launch_surr_pack_inf(c->s_wt, c->s_wi, s) != hipSuccess)
    return MPT_ERR_HIP;
  if (hipMemcpyAsync(c->s_bias, params + kOffB1, sizeof(float) * 128, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(c->s_bias + 128, params + kOffB2, sizeof(float) * 128, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(c->s_bias + 256, params + kOffB3, sizeof(float) * 128, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(c->s_bias + 384, params + kOffB4, sizeof(float) * 16, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(c->s_norm, norm, sizeof(float) * 12, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return MPT_ERR_HIP;
  c->s_tau = tau_km;
  c->s_loaded = 1;
  return MPT_OK;
}

namespace {
SurrW loaded_weights(const mpt_ctx *c) {
  SurrW W = surr_weights(c, nullptr, c->s_norm);
  W.b1 = c->s_bias;
  W.b2 = c->s_bias + 128;
  W.b3 = c->s_bias + 256;
  W.b4 = c->s_bias + 384;
  W.wi = c->s_wi;
  return W;
}
}  // namespace

mpt_status mpt_surrogate_forward(mpt_ctx *c, int64_t n, const float *x, float *y, void *hip_stream) {
  if (!c || n < 0 || (n > 0 && (!x || !y))) return MPT_ERR_ARG;
  if (!c->s_loaded) return MPT_ERR_STATE;
  if (n == 0) return MPT_OK;
  return from_hip(launch_surr_forward(loaded_weights(c), x, n, c->s_x, y, c->s_chunk,
                                     static_cast<hipStream_t>(hip_stream)));
}

mpt_status mpt_step_surrogate(mpt_ctx *c, mpt_particles *P, uint32_t step0, int32_t nsteps,
                              uint32_t *fallbacks, float *err_out, void *hip_stream) {
  if (!c || !fallbacks) return MPT_ERR_ARG;
  if (c->params.math != MPT_MATH_F32 || c->grid.dtype != MPT_DT_F32) return MPT_ERR_UNSUPPORTED;
  if (!P || P->scen) return MPT_ERR_UNSUPPORTED;
  if (c->params.flags & (MPT_CONV | MPT_SEDI)) return MPT_ERR_UNSUPPORTED;
  if (err_out && c->params.sort_interval > 0 && nsteps > 0) return MPT_ERR_ARG;  // fixed order needed
  if (step0 % kSurrK != 0 || nsteps < 0 || nsteps % kSurrK != 0) return MPT_ERR_ARG;
  if (!c->s_loaded) return MPT_ERR_STATE;
  const int S = c->params.sort_interval;
  mpt_status st = check_particles(c, P, S > 0 && nsteps > 0);
  if (st != MPT_OK) return st;
  if (P->n > 0 && (!P->up || !P->vp || !P->wp)) return MPT_ERR_ARG;
  st = check_time(c, step0, nsteps);
  if (st != MPT_OK) return st;
  if (P->n == 0 || nsteps == 0) return MPT_OK;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (P->n > c->n_max) return MPT_ERR_WORKSPACE;      // fallback list and sort keys hold n_max
  c->keyed = false;
  c->ordered = false;                                // the fallback list buffer is reused
  const SurrW W = loaded_weights(c);
  const int64_t end = (int64_t)step0 + nsteps;
  // a block sorts first when a multiple of sort_interval falls in it; the
  // block before such a block leaves the sort keys of its final positions
  // (apply for accepted and non-finite parcels, the plain steps for the rest)
  auto sort_due = [&](int64_t b) {
    for (int64_t q = b; S > 0 && q < b + kSurrK; ++q)
      if (q % S == 0) return true;
    return false;
  };
  bool keys_ready = false;
  for (int64_t b0 = step0; b0 < end; b0 += kSurrK) {
    if (sort_due(b0)) {
      st = do_sort(c, P, (uint32_t)b0, false, s, keys_ready);
      if (st != MPT_OK) return st;
    }
    const bool keys = b0 + kSurrK < end && sort_due(b0 + kSurrK);
    if (keys && launch_clear_spread(c->spread, (c->nkeys + 15) / 16, s) != hipSuccess) return MPT_ERR_HIP;
    StepArgs a;
    fill_step_args(c, P, (uint32_t)b0, kSurrK, c->params.flags, a);
    if (keys) a.sk = c->sk;
    if (launch_surr_tfield(a, c->params.t_start + (double)b0 * c->params.dt, c->s_f, s) != hipSuccess)
      return MPT_ERR_HIP;
    for (int64_t i0 = 0; i0 < P->n; i0 += c->s_chunk) {
      const int64_t cnt = P->n - i0 < c->s_chunk ? P->n - i0 : c->s_chunk;
      if (launch_surr_x(a, W, c->s_f, i0, cnt, c->s_x, c->s_chunk, s) != hipSuccess ||
          launch_surr_mlp(W, c->s_x, cnt, c->s_chunk, c->s_y, 4, s) != hipSuccess ||
          launch_surr_apply(a, c->s_tau, c->s_y, i0, cnt, err_out, c->fb_mask, s) != hipSuccess)
        return MPT_ERR_HIP;
    }
    if (launch_surr_fblist(c->fb_mask, P->n, c->fb_off, c->fb_sums, c->fb_list, fallbacks, s) != hipSuccess)
      return MPT_ERR_HIP;
    // parcels that fell back: kSurrK plain steps, walking the list
    StepArgs f;
    fill_step_args(c, P, (uint32_t)b0, kSurrK, c->params.flags, f);
    f.index = c->fb_list;
    f.index_count = c->fb_off + (P->n + 63) / 64;
    f.nblk = kPersistentBlocks;
    f.persistent = 1;
    if (keys) f.sk = c->sk;
    if (launch_step(c->grid.dtype, 0, f, s) != hipSuccess) return MPT_ERR_HIP;
    keys_ready = keys;
  }
  return MPT_OK;
}

mpt_status mpt_set_outgrid(mpt_ctx *c, const mpt_outgrid *g, void *hip_stream) {
  if (!c || !g || !g->pedges) return MPT_ERR_ARG;
  if (g->nx < 1 || g->ny < 1 || g->nz < 1 || g->nz > MPT_MAX_OUT_LEVELS) return MPT_ERR_ARG;
  if ((int64_t)g->nx * g->ny * g->nz > (int64_t)0x7FFFFFFF) return MPT_ERR_ARG;
  if (!(g->dlon > 0.0) || fabs(g->nx * g->dlon - 360.0) > 1e-9 || !isfinite(g->lon0)) return MPT_ERR_ARG;
  if (!(g->dlat > 0.0) || !(g->lat0 >= -90.0) || g->lat0 + g->ny * g->dlat > 90.0 + 1e-9) return MPT_ERR_ARG;
  for (int k = 0; k <= g->nz; ++k)
    if (!isfinite(g->pedges[k]) || (k > 0 && !(g->pedges[k] < g->pedges[k - 1]))) return MPT_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (hipMemcpyAsync(c->out_pe, g->pedges, sizeof(double) * (g->nz + 1), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return MPT_ERR_HIP;
  c->og = *g;
  c->og.pedges = c->out_pe;
  c->out_set = 1;
  return MPT_OK;
}

mpt_status mpt_grid_output(mpt_ctx *c, const mpt_particles *P, const double *mass, uint32_t *counts,
                           double *mass_sum, double *mmr, void *hip_stream) {
  if (!c || !P || !counts || !mass_sum || P->n < 0) return MPT_ERR_ARG;
  if (!aligned(counts, 4) || !aligned(mass_sum, 8) || (mmr && !aligned(mmr, 8))) return MPT_ERR_ARG;
  if (P->n > ((int64_t)1 << 31) * kBlock / 2) return MPT_ERR_UNSUPPORTED;
  if (P->n > 0) {
    if (!P->lon || !P->lat || !P->p) return MPT_ERR_ARG;
    if (!aligned(P->lon, 8) || !aligned(P->lat, 8) || !aligned(P->p, 8) || (mass && !aligned(mass, 8)))
      return MPT_ERR_ARG;
  }
  if (!c->out_set) return MPT_ERR_STATE;
  OutArgs o;
  o.lon = P->lon; o.lat = P->lat; o.p = P->p;
  o.mass = mass;
  o.n = P->n;
  o.nx = c->og.nx; o.ny = c->og.ny; o.nz = c->og.nz;
  o.lon0 = c->og.lon0; o.dlon = c->og.dlon; o.lat0 = c->og.lat0; o.dlat = c->og.dlat;
  o.pedges = c->out_pe;
  const int64_t nblk = (P->n + kOutParcelsPerBlock - 1) / kOutParcelsPerBlock;
  o.nblk = (int)nblk;
  o.per_xcd = (int)((nblk + kXcds - 1) / kXcds);
  return from_hip(launch_grid_out(o, counts, mass_sum, mmr, static_cast<hipStream_t>(hip_stream)));
}

mpt_status mpt_set_hybrid(mpt_ctx *c, int32_t nml, const double *a, const double *b, void *hip_stream) {
  if (!c || !a || !b || nml < 2 || nml > MPT_MAX_ML_LEVELS) return MPT_ERR_ARG;
  for (int k = 0; k < nml; ++k) {
    if (!isfinite(a[k]) || !isfinite(b[k])) return MPT_ERR_ARG;
    if (k > 0)
      for (double ps = 500.0; ps <= 1100.0; ps += 600.0)
        if (!(a[k] + b[k] * ps < a[k - 1] + b[k - 1] * ps)) return MPT_ERR_ARG;
    if (!(a[k] + b[k] * 500.0 > 0.0)) return MPT_ERR_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (hipMemcpyAsync(c->hyb_ab, a, sizeof(double) * nml, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(c->hyb_ab + nml, b, sizeof(double) * nml, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return MPT_ERR_HIP;
  c->hyb_nml = nml;
  return MPT_OK;
}

mpt_status mpt_ml_to_pl(mpt_ctx *c, const float *ps, const float *u, const float *v, const float *w,
                        float *u_pl, float *v_pl, float *w_pl, void *hip_stream) {
  if (!c || !ps || !u || !v || !w || !u_pl || !v_pl || !w_pl) return MPT_ERR_ARG;
  const float *ptrs[7] = {ps, u, v, w, u_pl, v_pl, w_pl};
  for (const float *q : ptrs)
    if (!aligned(q, 4)) return MPT_ERR_ARG;
  if (c->hyb_nml < 2) return MPT_ERR_STATE;
  Ml2PlArgs g;
  g.nx = c->grid.nx; g.ny = c->grid.ny; g.nz = c->grid.nz; g.nml = c->hyb_nml;
  g.plev = c->plev;
  g.a = c->hyb_ab;
  g.b = c->hyb_ab + c->hyb_nml;
  return from_hip(launch_ml_to_pl(g, ps, u, v, w, u_pl, v_pl, w_pl, static_cast<hipStream_t>(hip_stream)));
}

mpt_status mpt_destroy(mpt_ctx *c) {
  if (!c) return MPT_ERR_ARG;
  drop_graph(c);
  delete c;
  return MPT_OK;
}

const char *mpt_status_string(mpt_status s) {
  switch (s) {
    case MPT_OK: return "ok";
    case MPT_ERR_ARG: return "invalid argument";
    case MPT_ERR_STATE: return "invalid state (met level or release table not set)";
    case MPT_ERR_TIME: return "step outside the resident met time levels";
    case MPT_ERR_WORKSPACE: return "workspace too small or n > n_max";
    case MPT_ERR_HIP: return "HIP runtime error (or no GPU)";
    case MPT_ERR_UNSUPPORTED: return "unsupported combination";
  }
  return "unknown status";
}

}  // extern "C"
