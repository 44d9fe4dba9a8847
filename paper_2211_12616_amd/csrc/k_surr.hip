// k_surr.hip -- learned k-step advection surrogate (project addition; the
// paper has no counterpart): a ReLU MLP 81 -> 128 -> 128 -> 128 -> 3 on
// bf16 MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulate) that predicts the
// 8-step displacement of plain midpoint advection from u, v, w on the
// 3 x 3 x 3 cell stencil around the parcel.  Training data come from the
// plain scheme (FP64), training is hand-written forward / backward / Adam,
// and the step kernel falls back to 8 plain steps wherever a one-step
// midpoint consistency estimate of the prediction's error exceeds tau.
//
// Wave-level MLP: a wave runs 16-row tiles through the network; the A
// operand (activations) comes from LDS, the B operand (weights, [out][in]
// bf16, 16-byte fragments) from global memory, where the 94 KB of weights
// stay cache resident.
#include "mpt_device.h"
#include "mpt_internal.h"

namespace mpt {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t b = __float_as_uint(x);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t q) { return __uint_as_float((uint32_t)q << 16); }
__device__ __forceinline__ bf16x8 frag8(const uint16_t *p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(p));
}
__device__ __forceinline__ bf16x8 frag8_zero() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }
__device__ __forceinline__ bf16x8 frag8_strided(const uint16_t *p, int stride) {
  uint4 v;
  v.x = (uint32_t)p[0] | ((uint32_t)p[stride] << 16);
  v.y = (uint32_t)p[2 * stride] | ((uint32_t)p[3 * stride] << 16);
  v.z = (uint32_t)p[4 * stride] | ((uint32_t)p[5 * stride] << 16);
  v.w = (uint32_t)p[6 * stride] | ((uint32_t)p[7 * stride] << 16);
  return __builtin_bit_cast(bf16x8, v);
}
__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// One 16 x (16*nt) output tile: acc[nt] = A[16][K] . B[K][16] with A rows
// from LDS (stride lda), B given as [N][K] (stride K).  Lane l holds
// C[4*(l/16) + i][l%16] in acc[i].
template <class Epi>
__device__ __forceinline__ void gemm16(const uint16_t *a, int lda, int K, const uint16_t *bt, int N,
                                       Epi epi) {
  const int l = threadIdx.x & 63, row = l & 15, kq = l >> 4;
  for (int nt = 0; nt < N / 16; ++nt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < K / 32; ++kt)
      acc = mfma(frag8(a + row * lda + kt * 32 + kq * 8),
                 frag8(bt + (size_t)(nt * 16 + row) * K + kt * 32 + kq * 8), acc);
    epi(nt, kq, row, acc);
  }
}

// Hidden layer: out = relu(in . W + b) as bf16 into an LDS tile (and a copy
// to global rows when g is set).
__device__ __forceinline__ void dense_relu(const uint16_t *in, int ldi, int K, const uint16_t *wt,
                                           const float *b, uint16_t *out, uint16_t *g, int64_t g_row0,
                                           int64_t g_rows) {
  gemm16(in, ldi, K, wt, kSurrHid, [&](int nt, int kq, int row, f32x4 acc) {
    const float bias = b[nt * 16 + row];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint16_t v = f2bf(fmaxf(acc[i] + bias, 0.0f));
      const int m = kq * 4 + i;
      out[m * kHLd + nt * 16 + row] = v;
      if (g && g_row0 + m < g_rows) g[(g_row0 + m) * kSurrHid + nt * 16 + row] = v;
    }
  });
  __syncthreads();
}

// Output layer of one tile: normalized displacement, lane l holds
// rows 4*(l/16)+i of output column l%16 (columns >= 3 are padding).
__device__ __forceinline__ f32x4 dense_out(const uint16_t *in, const SurrW &W) {
  f32x4 r = {0.f, 0.f, 0.f, 0.f};
  gemm16(in, kHLd, kSurrHid, W.wt4, kSurrOutPad, [&](int, int, int row, f32x4 acc) {
    const float bias = W.b4[row];
#pragma unroll
    for (int i = 0; i < 4; ++i) r[i] = acc[i] + bias;
  });
  return r;
}

// Full network on one 16-row tile of normalized bf16 inputs xs (LDS).
__device__ __forceinline__ f32x4 mlp16(const uint16_t *xs, int ldx, const SurrW &W, uint16_t *ha,
                                       uint16_t *hb, uint16_t *g1, uint16_t *g2, uint16_t *g3,
                                       int64_t row0, int64_t rows) {
  dense_relu(xs, ldx, kSurrInPad, W.wt1, W.b1, ha, g1, row0, rows);
  dense_relu(ha, kHLd, kSurrHid, W.wt2, W.b2, hb, g2, row0, rows);
  dense_relu(hb, kHLd, kSurrHid, W.wt3, W.b3, ha, g3, row0, rows);
  return dense_out(ha, W);
}

// ---- stencil of the surrogate inputs -------------------------------------------
// u, v, w at the parcel position shifted by whole cells (a, b, c) in
// {-1, 0, 1} (lon, lat, level): quadrilinear interpolation of the shifted
// cell with the parcel's own weights, columns periodic, rows / levels
// clamped to valid cells.  Evaluated over the 4 x 4 x 4 points x 2 time
// levels around the cell; sink(idx, value), idx = var*27 + (c+1)*9 +
// (b+1)*3 + (a+1).
template <class Sink>
__device__ __forceinline__ void stencil81(const StepArgs &a, const Loc<float> &L, Sink sink) {
  const float4 *base = reinterpret_cast<const float4 *>(a.met);
  const float4 *lev0 = base + (int64_t)L.l * a.level_elems;
  const float4 *lev1 = lev0 + a.level_elems;
  int ic[4], jr[4], kr[4], pb[3], pc[3];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int ii = L.i0 - 1 + q;
    ii = ii < 0 ? ii + a.nx : (ii >= a.nx ? ii - a.nx : ii);
    ic[q] = ii;
    jr[q] = min(max(L.j - 1 + q, 0), a.ny - 1);
    kr[q] = min(max(L.k - 1 + q, 0), a.nz - 1);
  }
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    pb[s] = min(max(L.j - 1 + s, 0), a.ny - 2) - L.j + 1;   // row slot of shifted cell s-1
    pc[s] = min(max(L.k - 1 + s, 0), a.nz - 2) - L.k + 1;
  }
  float zprev[3][3][3], zcur[3][3][3];   // [b][a][var] at the previous / current level slot
#pragma unroll
  for (int qk = 0; qk < 4; ++qk) {
    float xprev[3][3], xcur[3][3];       // [a][var] at the previous / current row slot
#pragma unroll
    for (int qj = 0; qj < 4; ++qj) {
      const int64_t r = ((int64_t)kr[qk] * a.ny + jr[qj]) * a.nx;
      float v[4][3];
#pragma unroll
      for (int qi = 0; qi < 4; ++qi) {
        const float4 r0 = lev0[r + ic[qi]], r1 = lev1[r + ic[qi]];
        v[qi][0] = lerp(r0.x, r1.x, L.ft);
        v[qi][1] = lerp(r0.y, r1.y, L.ft);
        v[qi][2] = lerp(r0.z, r1.z, L.ft);
      }
#pragma unroll
      for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int q = 0; q < 3; ++q) xcur[s][q] = lerp(v[s][q], v[s + 1][q], L.fx);
      if (qj > 0) {
#pragma unroll
        for (int sb = 0; sb < 3; ++sb)
          if (pb[sb] + 1 == qj)
#pragma unroll
            for (int s = 0; s < 3; ++s)
#pragma unroll
              for (int q = 0; q < 3; ++q) zcur[sb][s][q] = lerp(xprev[s][q], xcur[s][q], L.fy);
      }
#pragma unroll
      for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int q = 0; q < 3; ++q) xprev[s][q] = xcur[s][q];
    }
    if (qk > 0) {
#pragma unroll
      for (int sc = 0; sc < 3; ++sc)
        if (pc[sc] + 1 == qk)
#pragma unroll
          for (int sb = 0; sb < 3; ++sb)
#pragma unroll
            for (int s = 0; s < 3; ++s)
#pragma unroll
              for (int q = 0; q < 3; ++q)
                sink(q * 27 + sc * 9 + sb * 3 + s, lerp(zprev[sb][s][q], zcur[sb][s][q], L.fz));
    }
#pragma unroll
    for (int sb = 0; sb < 3; ++sb)
#pragma unroll
      for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int q = 0; q < 3; ++q) zprev[sb][s][q] = zcur[sb][s][q];
  }
}

__device__ __forceinline__ void surr_locate(const StepArgs &a, double lon, double lat, double p,
                                            double t, Loc<float> &L) {
  locate_xyz<float>(a, a.plev, a.inv_dp, a.lut, lon, lat, p, L);
  locate_t<float>(a, t, L);
}

// ---- training data: stencil at the start, 8-step plain displacement ------------
__global__ __launch_bounds__(256) void k_surr_datagen(const StepArgs a, int64_t n, const double *lon,
                                                      const double *lat, const double *p,
                                                      const uint32_t *step, float *x, float *y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double lo = lon[i], la = lat[i], pp = p[i];
  const double t0 = a.t_start + (double)step[i] * a.dt;
  Loc<float> L;
  surr_locate(a, lo, la, pp, t0, L);
  float *xr = x + i * kSurrIn;
  stencil81(a, L, [&](int idx, float v) { xr[idx] = v; });
  double X = lo, Y = la, Z = pp;
  for (int q = 0; q < kSurrK; ++q) {
    advect<kF32, double>(a, a.plev, a.inv_dp, a.lut, t0 + (double)q * a.dt, X, Y, Z);
    position(a, X, Y, Z);
  }
  const double dl = fmod(X - lo + 540.0, 360.0) - 180.0;
  y[i * 3 + 0] = (float)(dl * kPi * kREarth * cos_floor<double>(a, la) / 180.0 / 1000.0);
  y[i * 3 + 1] = (float)((Y - la) * kPi * kREarth / 180.0 / 1000.0);
  y[i * 3 + 2] = (float)(Z - pp);
}

// ---- normalization statistics --------------------------------------------------
// Block b sums columns (81 inputs + 3 targets) over its chunk of samples.
__global__ __launch_bounds__(128) void k_surr_colsum(const float *x, const float *y, int64_t n,
                                                     double *part) {
  const int c = threadIdx.x;
  if (c >= kSurrIn + kSurrOut) return;
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t s0 = (int64_t)blockIdx.x * chunk, s1 = min(n, s0 + chunk);
  double s = 0.0, q = 0.0;
  for (int64_t i = s0; i < s1; ++i) {
    const double v = c < kSurrIn ? x[i * kSurrIn + c] : y[i * kSurrOut + (c - kSurrIn)];
    s += v;
    q += v * v;
  }
  part[((int64_t)blockIdx.x * 84 + c) * 2 + 0] = s;
  part[((int64_t)blockIdx.x * 84 + c) * 2 + 1] = q;
}

// norm = {in_mean[3], in_std[3], out_mean[3], out_std[3]}; input statistics
// pool the 27 stencil columns of each variable.
__global__ void k_surr_norm(const double *part, int nblk, int64_t n, float *norm) {
  __shared__ double cs[84][2];
  const int c = threadIdx.x;
  if (c < 84) {
    double s = 0.0, q = 0.0;
    for (int b = 0; b < nblk; ++b) {
      s += part[((int64_t)b * 84 + c) * 2];
      q += part[((int64_t)b * 84 + c) * 2 + 1];
    }
    cs[c][0] = s / (double)n;
    cs[c][1] = q / (double)n;
  }
  __syncthreads();
  if (c < 3) {
    double m = 0.0, q = 0.0;
    for (int k = 0; k < 27; ++k) {
      m += cs[c * 27 + k][0];
      q += cs[c * 27 + k][1];
    }
    m /= 27.0;
    q /= 27.0;
    norm[c] = (float)m;
    norm[3 + c] = (float)sqrt(fmax(q - m * m, 1e-30));
    const double om = cs[81 + c][0];
    norm[6 + c] = (float)om;
    norm[9 + c] = (float)sqrt(fmax(cs[81 + c][1] - om * om, 1e-30));
  }
}

// ---- parameters ----------------------------------------------------------------
struct LayerDims { int off_w, off_b, in_real, in_pad, out_real, out_pad; };
__device__ __forceinline__ LayerDims layer_dims(int l) {
  switch (l) {
    case 0: return {kOffW1, kOffB1, kSurrIn, kSurrInPad, kSurrHid, kSurrHid};
    case 1: return {kOffW2, kOffB2, kSurrHid, kSurrHid, kSurrHid, kSurrHid};
    case 2: return {kOffW3, kOffB3, kSurrHid, kSurrHid, kSurrHid, kSurrHid};
    default: return {kOffW4, kOffB4, kSurrHid, kSurrHid, kSurrOut, kSurrOutPad};
  }
}

// He-uniform weights U(-sqrt(6/fan_in), +) from Philox(index, 0, 3, 0); zero
// biases and zero padding rows / columns.
__global__ void k_surr_init(float *params, uint64_t seed) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kSurrNParam) return;
  for (int l = 0; l < 4; ++l) {
    const LayerDims d = layer_dims(l);
    const int nw = d.in_pad * d.out_pad;
    if (q >= d.off_w && q < d.off_w + nw) {
      const int r = (q - d.off_w) / d.out_pad, c = (q - d.off_w) % d.out_pad;
      float v = 0.0f;
      if (r < d.in_real && c < d.out_real) {
        uint32_t x[4];
        philox4x32_10((uint32_t)q, 0u, 3u, 0u, (uint32_t)seed, (uint32_t)(seed >> 32), x);
        const float u = ((float)(x[0] >> 8) + 0.5f) * (1.0f / 16777216.0f);
        v = (2.0f * u - 1.0f) * sqrtf(6.0f / (float)d.in_real);
      }
      params[q] = v;
      return;
    }
    if (q >= d.off_b && q < d.off_b + d.out_pad) {
      params[q] = 0.0f;
      return;
    }
  }
}

// bf16 copies: forward layout [out][in] for every layer, backward layout
// [in][out] for layers 2..4.
__global__ void k_surr_pack(const float *params, uint16_t *wt, uint16_t *wb) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  int acc_t = 0, acc_b = 0;
  for (int l = 0; l < 4; ++l) {
    const LayerDims d = layer_dims(l);
    const int nw = d.in_pad * d.out_pad;
    if (q < nw) {
      const int r = q / d.out_pad, c = q % d.out_pad;     // W[r = in][c = out]
      const uint16_t v = f2bf(params[d.off_w + q]);
      wt[acc_t + c * d.in_pad + r] = v;
      if (l > 0) wb[acc_b + q] = v;
    }
    acc_t += nw;
    if (l > 0) acc_b += nw;
  }
}

// ---- inference on given inputs (tests, calibration) ------------------------------
// One wave per 64 rows: raw inputs -> normalized bf16 tile -> MLP -> outputs
// de-normalized to (east km, north km, dp hPa).
__global__ __launch_bounds__(64) void k_surr_forward(const SurrW W, const float *x, int64_t n,
                                                     float *y) {
  __shared__ __attribute__((aligned(16))) uint16_t xs[64 * kXLd];
  __shared__ __attribute__((aligned(16))) uint16_t ha[16 * kHLd], hb[16 * kHLd];
  __shared__ float ys[64][4];
  const int l = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * 64, i = r0 + l;
  for (int c = 0; c < kXLd; ++c) {
    float v = 0.0f;
    if (i < n && c < kSurrIn) v = (x[i * kSurrIn + c] - W.norm[c / 27]) / W.norm[3 + c / 27];
    xs[l * kXLd + c] = f2bf(v);
  }
  __syncthreads();
  for (int t = 0; t < 4; ++t) {
    const f32x4 o = mlp16(xs + t * 16 * kXLd, kXLd, W, ha, hb, nullptr, nullptr, nullptr, 0, 0);
    const int row = l & 15, kq = l >> 4;
    if (row < kSurrOut)
#pragma unroll
      for (int q = 0; q < 4; ++q) ys[t * 16 + kq * 4 + q][row] = o[q];
    __syncthreads();
  }
  if (i < n)
    for (int q = 0; q < kSurrOut; ++q) y[i * kSurrOut + q] = W.norm[6 + q] + W.norm[9 + q] * ys[l][q];
}

// ---- training ---------------------------------------------------------------------
// Forward over a batch: one wave per 64 rows; keeps the normalized inputs,
// the three hidden activations (bf16) and the normalized outputs.
__global__ __launch_bounds__(64) void k_surr_train_fwd(const SurrW W, const SurrTrain T) {
  __shared__ __attribute__((aligned(16))) uint16_t xs[64 * kXLd];
  __shared__ __attribute__((aligned(16))) uint16_t ha[16 * kHLd], hb[16 * kHLd];
  const int l = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * 64, i = r0 + l;
  for (int c = 0; c < kXLd; ++c) {
    float v = 0.0f;
    if (c < kSurrIn) v = (T.x[i * kSurrIn + c] - W.norm[c / 27]) / W.norm[3 + c / 27];
    const uint16_t q = f2bf(v);
    xs[l * kXLd + c] = q;
    if (c < kSurrInPad) T.xn[i * kSurrInPad + c] = q;
  }
  __syncthreads();
  for (int t = 0; t < 4; ++t) {
    const int64_t tr = r0 + t * 16;
    const f32x4 o = mlp16(xs + t * 16 * kXLd, kXLd, W, ha, hb, T.h1, T.h2, T.h3, tr, T.batch);
    const int row = l & 15, kq = l >> 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) T.yp[(tr + kq * 4 + q) * kSurrOutPad + row] = o[q];
    __syncthreads();
  }
}

// Backward over a batch (one wave per 64 rows): loss gradient dY, then
// dH3 = dY W4^T, dH2 = dH3 W3^T, dH1 = dH2 W2^T, each masked by its ReLU.
__global__ __launch_bounds__(64) void k_surr_train_bwd(const SurrW W, const SurrTrain T) {
  __shared__ __attribute__((aligned(16))) uint16_t dy[16 * 40];
  __shared__ __attribute__((aligned(16))) uint16_t ga[16 * kHLd], gb[16 * kHLd];
  const int l = threadIdx.x, row = l & 15, kq = l >> 4;
  const float scale = 2.0f / (float)(kSurrOut * T.batch);
  float loss = 0.0f;
  for (int t = 0; t < 4; ++t) {
    const int64_t tr = (int64_t)blockIdx.x * 64 + t * 16;
    // dY tile: rows 4*kq+q, column row (K padded to 32 with zeros)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t r = tr + kq * 4 + q;
      float g = 0.0f;
      if (row < kSurrOut) {
        const float tn = (T.y[r * kSurrOut + row] - W.norm[6 + row]) / W.norm[9 + row];
        const float e = T.yp[r * kSurrOutPad + row] - tn;
        loss += e * e;
        g = scale * e;
      }
      const uint16_t gq = f2bf(g);
      dy[(kq * 4 + q) * 40 + row] = gq;
      dy[(kq * 4 + q) * 40 + 16 + row] = 0;
      T.dy[r * kSurrOutPad + row] = gq;
    }
    __syncthreads();
    // dH3 = dY . W4^T: B[k = out j][n = hidden i] = W4[i][j], [in][out] layout
    for (int nt = 0; nt < kSurrHid / 16; ++nt) {
      const int i = nt * 16 + row;
      const bf16x8 b = kq < 2 ? frag8(W.wb4 + i * kSurrOutPad + kq * 8) : frag8_zero();
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = mfma(frag8(dy + row * 40 + kq * 8), b, acc);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = tr + kq * 4 + q;
        const float h = bf2f(T.h3[r * kSurrHid + i]);
        const uint16_t g = f2bf(h > 0.0f ? acc[q] : 0.0f);
        ga[(kq * 4 + q) * kHLd + i] = g;
        T.dh3[r * kSurrHid + i] = g;
      }
    }
    __syncthreads();
    gemm16(ga, kHLd, kSurrHid, W.wb3, kSurrHid, [&](int nt, int kq_, int row_, f32x4 acc) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = tr + kq_ * 4 + q;
        const int i = nt * 16 + row_;
        const uint16_t g = f2bf(bf2f(T.h2[r * kSurrHid + i]) > 0.0f ? acc[q] : 0.0f);
        gb[(kq_ * 4 + q) * kHLd + i] = g;
        T.dh2[r * kSurrHid + i] = g;
      }
    });
    __syncthreads();
    gemm16(gb, kHLd, kSurrHid, W.wb2, kSurrHid, [&](int nt, int kq_, int row_, f32x4 acc) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = tr + kq_ * 4 + q;
        const int i = nt * 16 + row_;
        T.dh1[r * kSurrHid + i] = f2bf(bf2f(T.h1[r * kSurrHid + i]) > 0.0f ? acc[q] : 0.0f);
      }
    });
    __syncthreads();
  }
  // loss (reporting only): sum over the wave, one atomic per wave
  for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off);
  if (l == 0) atomicAdd(T.loss, loss / (float)(kSurrOut * T.batch));
}

// Weight gradients dW = A^T dH (reduction over the batch) for 16 x 16 tiles,
// one wave each; the last blocks sum bias gradients.
__global__ __launch_bounds__(64) void k_surr_wgrad(const SurrTrain T, float *grad) {
  const int l = threadIdx.x, row = l & 15, kq = l >> 4;
  int tile = blockIdx.x;
  // tiles per layer: 6x8, 8x8, 8x8, 8x1
  const int tiles[4] = {48, 64, 64, 8};
  int layer = 0;
  while (layer < 4 && tile >= tiles[layer]) tile -= tiles[layer++];
  if (layer == 4) {                       // bias gradients: 400 columns, 64 per block
    const int c = tile * 64 + l;
    const uint16_t *src;
    int ld, col, off;
    if (c < 128) { src = T.dh1; ld = kSurrHid; col = c; off = kOffB1; }
    else if (c < 256) { src = T.dh2; ld = kSurrHid; col = c - 128; off = kOffB2; }
    else if (c < 384) { src = T.dh3; ld = kSurrHid; col = c - 256; off = kOffB3; }
    else if (c < 400) { src = T.dy; ld = kSurrOutPad; col = c - 384; off = kOffB4; }
    else return;
    float s = 0.0f;
    for (int64_t r = 0; r < T.batch; ++r) s += bf2f(src[r * ld + col]);
    grad[off + col] = s;
    return;
  }
  const LayerDims d = layer_dims(layer);
  const int ntn = d.out_pad / 16;
  const int m0 = (tile / ntn) * 16, n0 = (tile % ntn) * 16;
  const uint16_t *A = layer == 0 ? T.xn : layer == 1 ? T.h1 : layer == 2 ? T.h2 : T.h3;
  const uint16_t *B = layer == 0 ? T.dh1 : layer == 1 ? T.dh2 : layer == 2 ? T.dh3 : T.dy;
  const int lda = layer == 0 ? kSurrInPad : kSurrHid;
  const int ldb = layer == 3 ? kSurrOutPad : kSurrHid;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int64_t b0 = 0; b0 < T.batch; b0 += 32) {
    const int64_t r = b0 + kq * 8;
    acc = mfma(frag8_strided(A + r * lda + m0 + row, lda), frag8_strided(B + r * ldb + n0 + row, ldb), acc);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) grad[d.off_w + (m0 + kq * 4 + q) * d.out_pad + n0 + row] = acc[q];
}

__global__ void k_surr_adam(float *params, const float *grad, float *m, float *v, float lr, float bc1,
                            float bc2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kSurrNParam) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float g = grad[q];
  const float mq = b1 * m[q] + (1.0f - b1) * g;
  const float vq = b2 * v[q] + (1.0f - b2) * g * g;
  m[q] = mq;
  v[q] = vq;
  params[q] -= lr * (mq / bc1) / (sqrtf(vq / bc2) + eps);
}

// ---- surrogate stepping -------------------------------------------------------------
// One wave per 64 parcels, one block of kSurrK steps from step0:
// stencil -> MLP -> consistency estimate -> accept (displacement plus the
// block's turbulent and mesoscale diffusion with the block-start spread) or
// kSurrK plain steps.
__global__ __launch_bounds__(64) void k_surr_step(const StepArgs a, const SurrW W, float tau_km,
                                                  uint32_t *fallbacks, float *err_out,
                                                  uint32_t *fb_list, uint32_t *fb_count) {
  __shared__ __attribute__((aligned(16))) uint16_t xs[64 * kXLd];
  __shared__ __attribute__((aligned(16))) uint16_t ha[16 * kHLd], hb[16 * kHLd];
  __shared__ float ys[64][4];
  const int l = threadIdx.x;
  const int lb = logical_block((int)blockIdx.x, a.per_xcd);
  if (lb >= a.nblk) return;
  const int64_t i = (int64_t)lb * 64 + l;
  const bool in_range = i < a.n;
  double lon = 0.0, lat = 0.0, p = 500.0;
  if (in_range) {
    lon = a.lon[i];
    lat = a.lat[i];
    p = a.p[i];
  }
  const bool valid = in_range && finite3(lon, lat, p);
  const double t0 = a.t_start + (double)a.step0 * a.dt;
  Loc<float> L;
  surr_locate(a, valid ? lon : 0.0, valid ? lat : 0.0, valid ? p : 500.0, t0, L);
  stencil81(a, L, [&](int idx, float v) {
    xs[l * kXLd + idx] = f2bf((v - W.norm[idx / 27]) / W.norm[3 + idx / 27]);
  });
  for (int c = kSurrIn; c < kXLd; ++c) xs[l * kXLd + c] = 0;
  __syncthreads();
  for (int t = 0; t < 4; ++t) {
    const f32x4 o = mlp16(xs + t * 16 * kXLd, kXLd, W, ha, hb, nullptr, nullptr, nullptr, 0, 0);
    const int row = l & 15, kq = l >> 4;
    if (row < kSurrOut)
#pragma unroll
      for (int q = 0; q < 4; ++q) ys[t * 16 + kq * 4 + q][row] = o[q];
    __syncthreads();
  }
  if (!valid) return;
  const float de = W.norm[6] + W.norm[9] * ys[l][0];
  const float dn = W.norm[7] + W.norm[10] * ys[l][1];
  const float dpp = W.norm[8] + W.norm[11] * ys[l][2];
  // consistency estimate: kSurrK dt times the wind at the predicted midpoint
  const float c0 = cos_floor<float>(a, lat);
  const float kdeg = (float)kDeg;
  const double lonm = lon + (double)(0.5f * de * 1000.0f * kdeg / c0);
  const double latm = lat + (double)(0.5f * dn * 1000.0f * kdeg);
  const double pm = p + (double)(0.5f * dpp);
  Cell16<kF32> cell;
  Loc<float> Lm;
  surr_locate(a, lonm, latm, pm, t0 + 0.5 * kSurrK * a.dt, Lm);
  load_cell<kF32, float>(a, Lm, cell);
  float wm[3];
  interp_cell<kF32, float>(a, cell, Lm, wm);
  const float span = (float)(kSurrK * a.dt) * 1e-3f;
  const float ee = de - span * wm[0], en = dn - span * wm[1];
  const float err = sqrtf(ee * ee + en * en);
  if (err_out) err_out[i] = err;
  const uint32_t id = a.id[i];
  float up = static_cast<const float *>(a.up)[i];
  float vp = static_cast<const float *>(a.vp)[i];
  float wp = static_cast<const float *>(a.wp)[i];
  const bool meso_on = (a.flags & kMeso) != 0;
  const bool accept = err <= tau_km && isfinite(err);
  // parcels that fall back keep their state here and are queued for the
  // plain step kernel (a wave-aggregated append to the list)
  const uint64_t fb = __ballot(!accept);
  if (fb) {
    const int leader = __ffsll((long long)fb) - 1;
    uint32_t base = 0;
    if (l == leader) {
      base = atomicAdd(fb_count, (uint32_t)__popcll(fb));
      atomicAdd(fallbacks, (uint32_t)__popcll(fb));
    }
    base = __shfl(base, leader);
    if (!accept) fb_list[base + __popcll(fb & ((1ull << l) - 1ull))] = (uint32_t)i;
  }
  if (!accept) return;
  float sg[3] = {0.f, 0.f, 0.f};
  if (meso_on) meso_sigma<kF32, float>(a, a.plev, a.inv_dp, a.lut, t0 + 0.5 * a.dt, lon, lat, p, sg);
  lon = lon + (double)(de * 1000.0f * kdeg / c0);
  lat = lat + (double)(dn * 1000.0f * kdeg);
  p = p + (double)dpp;
  position(a, lon, lat, p);
  for (int s = 0; s < kSurrK; ++s) {
    const uint32_t step = a.step0 + (uint32_t)s;
    if (a.flags & kTurb) turb<float>(a, id, step, lon, lat, p);
    if (meso_on) {
      float xi[3];
      normals3<float>(a.seed, id, step, 1u, xi);
      meso_apply<float>(a, sg, xi, lon, lat, p, up, vp, wp);
    }
    position(a, lon, lat, p);
  }
  a.lon[i] = lon;
  a.lat[i] = lat;
  a.p[i] = p;
  static_cast<float *>(a.up)[i] = up;
  static_cast<float *>(a.vp)[i] = vp;
  static_cast<float *>(a.wp)[i] = wp;
}

// ---- launchers ------------------------------------------------------------------------
hipError_t launch_surr_datagen(const StepArgs &a, int64_t n, const double *lon, const double *lat,
                               const double *p, const uint32_t *step, float *x, float *y,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_surr_datagen, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, n, lon, lat,
                     p, step, x, y);
  return hipGetLastError();
}

hipError_t launch_surr_stats(const float *x, const float *y, int64_t n, double *part, int nblk,
                             float *norm, hipStream_t s) {
  hipLaunchKernelGGL(k_surr_colsum, dim3((unsigned)nblk), dim3(128), 0, s, x, y, n, part);
  hipLaunchKernelGGL(k_surr_norm, dim3(1), dim3(128), 0, s, part, nblk, n, norm);
  return hipGetLastError();
}

hipError_t launch_surr_init(float *params, uint64_t seed, hipStream_t s) {
  hipLaunchKernelGGL(k_surr_init, dim3((kSurrNParam + 255) / 256), dim3(256), 0, s, params, seed);
  return hipGetLastError();
}

hipError_t launch_surr_pack(const float *params, uint16_t *wt, uint16_t *wb, hipStream_t s) {
  hipLaunchKernelGGL(k_surr_pack, dim3((kSurrHid * kSurrHid + 255) / 256), dim3(256), 0, s, params, wt, wb);
  return hipGetLastError();
}

hipError_t launch_surr_forward(const SurrW &W, const float *x, int64_t n, float *y, hipStream_t s) {
  hipLaunchKernelGGL(k_surr_forward, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, W, x, n, y);
  return hipGetLastError();
}

hipError_t launch_surr_train(const SurrW &W, const SurrTrain &T, float *params, float *m, float *v,
                             float lr, float bc1, float bc2, hipStream_t s) {
  const unsigned nb = (unsigned)(T.batch / 64);
  hipLaunchKernelGGL(k_surr_train_fwd, dim3(nb), dim3(64), 0, s, W, T);
  hipLaunchKernelGGL(k_surr_train_bwd, dim3(nb), dim3(64), 0, s, W, T);
  hipLaunchKernelGGL(k_surr_wgrad, dim3(48 + 64 + 64 + 8 + 7), dim3(64), 0, s, T, T.grad);
  hipLaunchKernelGGL(k_surr_adam, dim3((kSurrNParam + 255) / 256), dim3(256), 0, s, params, T.grad, m, v,
                     lr, bc1, bc2);
  return hipGetLastError();
}

hipError_t launch_surr_grad(const SurrW &W, const SurrTrain &T, hipStream_t s) {
  const unsigned nb = (unsigned)(T.batch / 64);
  hipLaunchKernelGGL(k_surr_train_fwd, dim3(nb), dim3(64), 0, s, W, T);
  hipLaunchKernelGGL(k_surr_train_bwd, dim3(nb), dim3(64), 0, s, W, T);
  hipLaunchKernelGGL(k_surr_wgrad, dim3(48 + 64 + 64 + 8 + 7), dim3(64), 0, s, T, T.grad);
  return hipGetLastError();
}

hipError_t launch_surr_step(const StepArgs &a, const SurrW &W, float tau_km, uint32_t *fallbacks,
                            float *err_out, uint32_t *fb_list, uint32_t *fb_count, hipStream_t s) {
  hipLaunchKernelGGL(k_surr_step, dim3((unsigned)(a.per_xcd * kXcds)), dim3(64), 0, s, a, W, tau_km,
                     fallbacks, err_out, fb_list, fb_count);
  return hipGetLastError();
}

}  // namespace mpt
