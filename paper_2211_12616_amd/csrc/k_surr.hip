// k_surr.hip -- learned k-step advection surrogate (project addition; the
// paper has no counterpart): a ReLU MLP 81 -> 128 -> 128 -> 128 -> 3 on
// bf16 MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulate) that predicts the
// 8-step displacement of plain midpoint advection from u, v, w on the
// 3 x 3 x 3 cell stencil around the parcel.  Training data come from the
// plain scheme (FP64), training is hand-written forward / backward / Adam,
// and the step kernel falls back to 8 plain steps wherever a one-step
// midpoint consistency estimate of the prediction's error exceeds tau.
//
// Inference (k_surr_mlp) is a persistent kernel, one block per CU, that
// stages the 94 KB of bf16 weights in LDS once and keeps the activations in
// registers (transposed products, below).  Training runs 16-row tiles with
// the activations in LDS and the weights read from global memory.
#include "mpt_device.h"
#include "mpt_internal.h"
#include "mpt_stage.h"

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
// levels around the cell.  The values of one level shift c come out
// together, in ascending c: sink(c + 1, g) with g[(b+1)*9 + (a+1)*3 + var];
// the input index of a value is var*27 + (c+1)*9 + (b+1)*3 + (a+1).
// The values of grid point (k, j, i) come from src(k, j, i, v): the
// time-interpolated field (global memory or an LDS box) or the two met
// levels of L interpolated in time on the spot.
template <class Src, class Sink>
__device__ __forceinline__ void stencil81(const StepArgs &a, const Loc<float> &L, Src src, Sink sink) {
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
      float v[4][3];
#pragma unroll
      for (int qi = 0; qi < 4; ++qi) src(kr[qk], jr[qj], ic[qi], v[qi]);
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
        if (pc[sc] + 1 == qk) {
          float g[27];
#pragma unroll
          for (int sb = 0; sb < 3; ++sb)
#pragma unroll
            for (int s = 0; s < 3; ++s)
#pragma unroll
              for (int q = 0; q < 3; ++q) g[sb * 9 + s * 3 + q] = lerp(zprev[sb][s][q], zcur[sb][s][q], L.fz);
          sink(sc, g);
        }
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
  locate_xyz_g<float>(a, lon, lat, p, L);
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
  const float4 *lev0 = reinterpret_cast<const float4 *>(a.met) + (int64_t)L.l * a.level_elems;
  const float4 *lev1 = reinterpret_cast<const float4 *>(a.met) + (int64_t)L.l1 * a.level_elems;
  auto src = [&](int k, int j, int ii, float (&v)[3]) {
    const int64_t q = ((int64_t)k * a.ny + j) * a.nx + ii;
    const float4 r0 = lev0[q], r1 = lev1[q];
    v[0] = lerp(r0.x, r1.x, L.ft);
    v[1] = lerp(r0.y, r1.y, L.ft);
    v[2] = lerp(r0.z, r1.z, L.ft);
  };
  stencil81(a, L, src, [&](int sc, const float (&g)[27]) {
#pragma unroll
    for (int j = 0; j < 27; ++j) xr[(j % 3) * 27 + sc * 9 + j / 3] = g[j];
  });
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

// ---- inference: persistent MLP with the weights in LDS --------------------------------
// Each layer computes H^T = W^T X^T: the weights are the A operand (rows =
// output units) and 16 parcels are the columns of B, so the accumulator
// tiles of one layer (lane l: units 4*(l/16)+i of parcel l%16) are already
// the B fragments of the next once the K order of the next layer's weights
// is permuted to match: slot (kt, g, j) of a 32-wide K tile holds unit
// 32 kt + 4 g + j for j < 4 and 32 kt + 16 + 4 g + j - 4 for j >= 4.
// Activations never leave registers; every weight fragment read from LDS
// serves the 4 parcel tiles of a wave.
constexpr int kMlpThreads = 512;
constexpr int kMlpBlocks = 256;                               // one per CU

typedef __attribute__((__vector_size__(8 * sizeof(float)))) float f32x8;

__device__ __forceinline__ float relu_bits(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

// relu, then bf16 (round to nearest even) of 4 + 4 accumulator values
__device__ __forceinline__ bf16x8 pack_relu(const f32x4 &a, const f32x4 &b) {
  const f32x8 v = {relu_bits(a[0]), relu_bits(a[1]), relu_bits(a[2]), relu_bits(a[3]),
                   relu_bits(b[0]), relu_bits(b[1]), relu_bits(b[2]), relu_bits(b[3])};
  return __builtin_convertvector(v, bf16x8);
}

// One hidden layer over the wave's 4 parcel tiles: in[t][kt] (KT K tiles)
// -> out[t][p], p = the next layer's K tile (m-tiles 2p and 2p + 1).
template <int KT>
__device__ __forceinline__ void mlp_layer(const uint16_t *sw, int ld, const float *sbias,
                                          const bf16x8 (&in)[4][KT], bf16x8 (&out)[4][4]) {
  const int l = threadIdx.x & 63, col = l & 15, g = l >> 4;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    f32x4 acc[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int mt = 2 * p + h;
      const f32x4 b = *reinterpret_cast<const f32x4 *>(sbias + 16 * mt + 4 * g);
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[h][t] = b;
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) {
        const bf16x8 a = frag8(sw + (16 * mt + col) * ld + 32 * kt + 8 * g);
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[h][t] = mfma(a, in[t][kt], acc[h][t]);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) out[t][p] = pack_relu(acc[0][t], acc[1][t]);
  }
}

// Stencil rows in the MLP's input order: K tile c (32 wide) holds the 27
// values of level shift c - 1 as (b, a, var) with var fastest, then 5 zeros
// (input index of slot j < 27: (j % 3) * 27 + c * 9 + j / 3).  The
// layer-1 weights are permuted to this order when they are staged.
__device__ __forceinline__ void pack_ktile(const float (&g)[27], const float (&inv)[3], const float *norm,
                                           bf16x8 (&dst)[4]) {
#pragma unroll
  for (int c8 = 0; c8 < 4; ++c8) {
    f32x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int q = 8 * c8 + j;
      v[j] = q < 27 ? (g[q] - norm[q % 3]) * inv[q % 3] : 0.0f;
    }
    dst[c8] = __builtin_convertvector(v, bf16x8);
  }
}

// Stencil rows in global memory, chunk-major: the 16-byte chunk c (inputs
// 8c .. 8c + 7 in the order above) of row r is at X + (c * ldc + r) * 8, so
// that a wave's stores of one chunk of 64 consecutive rows are contiguous.
__device__ __forceinline__ uint16_t *x_chunk(uint16_t *X, int64_t ldc, int c, int64_t r) {
  return X + ((int64_t)c * ldc + r) * 8;
}
__device__ __forceinline__ const uint16_t *x_chunk(const uint16_t *X, int64_t ldc, int c, int64_t r) {
  return X + ((int64_t)c * ldc + r) * 8;
}

// K tile sc of row r: chunks 4 sc .. 4 sc + 3.  The chunk bases are
// uniform and the row's byte offset (r < 2^28) is shared by the four
// stores.
__device__ __forceinline__ void store_ktile(const float (&g)[27], const float (&inv)[3], const float *norm,
                                            uint16_t *X, int64_t ldc, int sc, int64_t r) {
  bf16x8 t[4];
  pack_ktile(g, inv, norm, t);
  const size_t roff = (size_t)((uint32_t)r * 16u);
#pragma unroll
  for (int c8 = 0; c8 < 4; ++c8)
    *reinterpret_cast<bf16x8 *>(reinterpret_cast<char *>(x_chunk(X, ldc, 4 * sc + c8, 0)) + roff) = t[c8];
}

// The inference LDS image of the forward weights wt: layer 1 with K in the
// stencil rows' order (slot 32 c + j < 32 c + 27 of row m holds input
// (j % 3) * 27 + c * 9 + j / 3), layers 2..4 with K in the order of the
// accumulator tiles of the layer before (slot 32 kt + 8 g + j holds unit
// 32 kt + 4 g + j for j < 4, 32 kt + 16 + 4 g + j - 4 for j >= 4); rows
// padded by 8 zeros against LDS bank conflicts.
__global__ void k_surr_pack_inf(const uint16_t *wt, uint16_t *wi) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kWiSize) return;
  uint16_t v = 0;
  if (e < kSurrHid * kW1Ld) {
    const int m = e / kW1Ld, k = e % kW1Ld, c = k >> 5, j = k & 31;
    if (k < kSurrInPad && j < 27) v = wt[m * kSurrInPad + (j % 3) * 27 + c * 9 + j / 3];
  } else {
    const int e2 = e - kSurrHid * kW1Ld;
    const int layer = e2 / (kSurrHid * kWLd);             // 0, 1: W2, W3; 2: W4
    const int m = (e2 % (kSurrHid * kWLd)) / kWLd, k = e2 % kWLd;
    const uint16_t *src = wt + kSurrHid * kSurrInPad + layer * kSurrHid * kSurrHid;
    if (k < kSurrHid) {
      const int kt = k >> 5, g = (k >> 3) & 3, j = k & 7;
      v = src[m * kSurrHid + 32 * kt + (j < 4 ? 4 * g + j : 16 + 4 * g + j - 4)];
    }
  }
  wi[e] = v;
}

// Persistent over groups of 64 parcels: X rows (bf16, normalized, 96 wide,
// chunk-major with ldc rows per chunk) -> Y[row * ldy + q] = de-normalized
// (east km, north km, dp hPa).
__global__ __launch_bounds__(kMlpThreads) void k_surr_mlp(const SurrW W, const uint16_t *X, int64_t n,
                                                          int64_t ldc, float *Y, int ldy) {
  __shared__ __attribute__((aligned(16))) uint16_t sw[kWiSize];
  __shared__ __attribute__((aligned(16))) float sb[3 * kSurrHid + kSurrOutPad + 12];
  uint16_t *sw1 = sw, *sw2 = sw1 + kSurrHid * kW1Ld, *sw3 = sw2 + kSurrHid * kWLd, *sw4 = sw3 + kSurrHid * kWLd;
  const int tid = threadIdx.x;
  for (int q = tid; q < kWiSize / 8; q += kMlpThreads)
    reinterpret_cast<uint4 *>(sw)[q] = reinterpret_cast<const uint4 *>(W.wi)[q];
  for (int q = tid; q < kSurrHid; q += kMlpThreads) {
    sb[q] = W.b1[q];
    sb[kSurrHid + q] = W.b2[q];
    sb[2 * kSurrHid + q] = W.b3[q];
  }
  if (tid < kSurrOutPad) sb[3 * kSurrHid + tid] = W.b4[tid];
  if (tid < 12) sb[3 * kSurrHid + kSurrOutPad + tid] = W.norm[tid];
  __syncthreads();
  const float *nm = sb + 3 * kSurrHid + kSurrOutPad;
  const int l = tid & 63, col = l & 15, g = l >> 4;
  constexpr int kWaves = kMlpThreads / 64;
  const int64_t ngroups = (n + 63) / 64;
  for (int64_t grp = (int64_t)blockIdx.x * kWaves + (tid >> 6); grp < ngroups;
       grp += (int64_t)gridDim.x * kWaves) {
    // keeps the weight fragment reads inside the loop (hoisted, the 92
    // fragments would need 368 registers)
    asm volatile("" ::: "memory");
    bf16x8 x[4][kSurrInPad / 32];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t row = grp * 64 + 16 * t + col;
#pragma unroll
      for (int kt = 0; kt < kSurrInPad / 32; ++kt)
        x[t][kt] = row < n ? frag8(x_chunk(X, ldc, 4 * kt + g, row)) : frag8_zero();
    }
    bf16x8 h1[4][4], h2[4][4];
    mlp_layer<kSurrInPad / 32>(sw1, kW1Ld, sb, x, h1);
    mlp_layer<4>(sw2, kWLd, sb + kSurrHid, h1, h2);
    mlp_layer<4>(sw3, kWLd, sb + 2 * kSurrHid, h2, h1);
    f32x4 o[4];
    const f32x4 b4 = *reinterpret_cast<const f32x4 *>(sb + 3 * kSurrHid + 4 * g);
#pragma unroll
    for (int t = 0; t < 4; ++t) o[t] = b4;
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
      const bf16x8 a = frag8(sw4 + col * kWLd + 32 * kt + 8 * g);
#pragma unroll
      for (int t = 0; t < 4; ++t) o[t] = mfma(a, h1[t][kt], o[t]);
    }
    if (g == 0) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t row = grp * 64 + 16 * t + col;
        if (row < n)
#pragma unroll
          for (int q = 0; q < kSurrOut; ++q) Y[row * ldy + q] = nm[6 + q] + nm[9 + q] * o[t][q];
      }
    }
  }
}

// Raw inputs (FP32, 81 per row, input index order) -> normalized bf16 rows
// of 96 in the MLP's input order, chunk-major (see store_ktile).
__global__ __launch_bounds__(256) void k_surr_xnorm(const SurrW W, const float *x, int64_t n,
                                                    uint16_t *X, int64_t ldc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float inv[3];
#pragma unroll
  for (int v = 0; v < 3; ++v) inv[v] = 1.0f / W.norm[3 + v];
  const float *xr = x + i * kSurrIn;
#pragma unroll
  for (int sc = 0; sc < 3; ++sc) {
    float g[27];
#pragma unroll
    for (int j = 0; j < 27; ++j) g[j] = xr[(j % 3) * 27 + sc * 9 + j / 3];
    store_ktile(g, inv, W.norm, X, ldc, sc, i);
  }
}

// ---- training ---------------------------------------------------------------------
// Forward over a batch: one wave per 64 rows; keeps the normalized inputs,
// the three hidden activations (bf16) and the normalized outputs.
__global__ __launch_bounds__(64) void k_surr_train_fwd(const SurrW W, const SurrTrain T) {
  __shared__ __attribute__((aligned(16))) uint16_t xs[64 * kXLd];
  __shared__ __attribute__((aligned(16))) uint16_t ha[16 * kHLd], hb[16 * kHLd];
  const int l = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * 64, i = r0 + l;
  float inv[3];
#pragma unroll
  for (int v = 0; v < 3; ++v) inv[v] = 1.0f / W.norm[3 + v];
  for (int c = 0; c < kXLd; ++c) {
    float v = 0.0f;
    if (c < kSurrIn) v = (T.x[i * kSurrIn + c] - W.norm[c / 27]) * inv[c / 27];
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
// one wave per tile and share of the batch (blockIdx.y of gridDim.y shares
// of its 32-row chunks), added into grad (zeroed before); the last blocks
// sum bias gradients the same way.
__global__ __launch_bounds__(64) void k_surr_wgrad(const SurrTrain T, float *grad) {
  const int l = threadIdx.x, row = l & 15, kq = l >> 4;
  const int64_t nch = T.batch / 32;
  const int64_t r_lo = 32 * (nch * blockIdx.y / gridDim.y), r_hi = 32 * (nch * (blockIdx.y + 1) / gridDim.y);
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
    for (int64_t r = r_lo; r < r_hi; ++r) s += bf2f(src[r * ld + col]);
    atomicAdd(&grad[off + col], s);
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
  for (int64_t b0 = r_lo; b0 < r_hi; b0 += 32) {
    const int64_t r = b0 + kq * 8;
    acc = mfma(frag8_strided(A + r * lda + m0 + row, lda), frag8_strided(B + r * ldb + n0 + row, ldb), acc);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) atomicAdd(&grad[d.off_w + (m0 + kq * 4 + q) * d.out_pad + n0 + row], acc[q]);
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
// A block of kSurrK steps runs over chunks of parcels in three passes:
// stencil rows (k_surr_x), MLP (k_surr_mlp), then the consistency estimate
// and either acceptance (displacement plus the block's turbulent and
// mesoscale diffusion with the plain steps' draws and the block-start
// spread) or a place in the list of parcels that take kSurrK plain steps
// (k_surr_apply).

// The FP32 field at time t (all points): F = lerp(level l, level l + 1, ft)
// per component with the (l, ft) a parcel at time t computes.
__global__ __launch_bounds__(256) void k_surr_tfield(const StepArgs a, double t, float4 *F) {
  Loc<float> L;
  locate_t<float>(a, t, L);
  const float4 *lev0 = reinterpret_cast<const float4 *>(a.met) + (int64_t)L.l * a.level_elems;
  const float4 *lev1 = reinterpret_cast<const float4 *>(a.met) + (int64_t)L.l1 * a.level_elems;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < a.level_elems;
       q += (int64_t)gridDim.x * blockDim.x) {
    const float4 r0 = lev0[q], r1 = lev1[q];
    F[q] = make_float4(lerp(r0.x, r1.x, L.ft), lerp(r0.y, r1.y, L.ft), lerp(r0.z, r1.z, L.ft), 0.0f);
  }
}

// Stencil inputs of parcels i0 .. i0 + cnt - 1 at the block's start time,
// normalized, as bf16 rows of 96 in the MLP's input order, chunk-major with
// ldc rows per chunk (x_chunk); a parcel with a non-finite position gets a
// zero row.  The block's 256 parcels (sorted by tile) read their 4 x 4 x 4
// stencil points from an LDS box: the bounding box of their cells
// (mpt_stage.h) widened by one point below and two above in each direction
// (rows and levels clamped to the grid), loaded from the field at the
// block's start time with coalesced loads; a box that does not fit makes
// the block read the points from global memory.  Each lane stores its own
// row; a wave's store of one chunk covers 64 consecutive rows.
constexpr int kSurrBoxCap = 1536;               // grid points of the stencil box

__global__ __launch_bounds__(256) void k_surr_x(const StepArgs a, const SurrW W, const float4 *F,
                                                int64_t i0, int64_t cnt, uint16_t *X, int64_t ldc) {
  __shared__ float bu[kSurrBoxCap], bv[kSurrBoxCap], bw[kSurrBoxCap];
  __shared__ __attribute__((aligned(16))) int red[kRedInts];
  const int lb = logical_block((int)blockIdx.x, a.per_xcd);
  if (lb >= a.nblk) return;                       // uniform over the block
  const int64_t r0 = (int64_t)lb * 256;
  const int64_t r = r0 + threadIdx.x;
  bool valid = false;
  double lon = 0.0, lat = 0.0, p = 0.0;
  if (r < cnt) {
    lon = a.lon[i0 + r];
    lat = a.lat[i0 + r];
    p = a.p[i0 + r];
    valid = finite3(lon, lat, p);
  }
  Loc<float> L;
  surr_locate(a, lon, lat, p, a.t_start + (double)a.step0 * a.dt, L);
  StepLds<float> sm;
  sm.red = red;
  BoxRef ref = block_ref(a, a.plev, a.lut, i0 + r0, true);
  const Box b = block_box<float>(a, sm, valid, L, ref);
  // stencil points of the box's cells
  int gs = b.gi - 1;
  if (gs < 0) gs += a.nx;
  const int ni = b.bi + 2;
  const int js = max(b.j0 - 1, 0), ks = max(b.k0 - 1, 0);
  const int nj = min(b.j0 + b.bj, a.ny - 1) - js + 1, nk = min(b.k0 + b.bk, a.nz - 1) - ks + 1;
  const bool staged = ni <= a.nx && ni <= kMaxExtent && nj <= kMaxExtent && ni * nj * nk <= kSurrBoxCap;
  if (staged) {
    const int npts = ni * nj * nk;
    const uint32_t mi = kDivMagic.m[ni], mj = kDivMagic.m[nj];
    // four points per thread and pass, all loads issued before the stores;
    // a clamped duplicate of the last point rewrites that point's own value
    for (int q0 = (int)threadIdx.x; q0 < npts; q0 += 4 * 256) {
      float4 v[4];
      int qq[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = min(q0 + u * 256, npts - 1);
        qq[u] = q;
        const int rr = (int)__umulhi((uint32_t)q, mi);
        const int ii = q - rr * ni;
        const int kk = (int)__umulhi((uint32_t)rr, mj);
        const int jj = rr - kk * nj;
        int gi = gs + ii;
        if (gi >= a.nx) gi -= a.nx;
        v[u] = F[((ks + kk) * a.ny + js + jj) * a.nx + gi];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        bu[qq[u]] = v[u].x;
        bv[qq[u]] = v[u].y;
        bw[qq[u]] = v[u].z;
      }
    }
  }
  __syncthreads();
  if (r >= cnt) return;                           // no barrier follows
  if (valid) {
    float inv[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) inv[v] = 1.0f / W.norm[3 + v];
    auto sink = [&](int sc, const float (&g)[27]) { store_ktile(g, inv, W.norm, X, ldc, sc, r); };
    if (staged) {
      auto src = [&](int k, int j, int ii, float (&v)[3]) {
        int li = ii - gs;
        if (li < 0) li += a.nx;
        const int q = ((k - ks) * nj + (j - js)) * ni + li;
        v[0] = bu[q];
        v[1] = bv[q];
        v[2] = bw[q];
      };
      stencil81(a, L, src, sink);
    } else {
      // blocks whose box does not fit (rare): the loads stay in program
      // order (the empty asm), so the fallback does not hoist a whole
      // level's loads and set the register budget of the kernel
      auto src = [&](int k, int j, int ii, float (&v)[3]) {
        asm volatile("" ::: "memory");
        const float4 f = F[((int64_t)k * a.ny + j) * a.nx + ii];
        v[0] = f.x;
        v[1] = f.y;
        v[2] = f.z;
      };
      stencil81(a, L, src, sink);
    }
  } else {
#pragma unroll
    for (int c = 0; c < kSurrInPad / 8; ++c)
      *reinterpret_cast<bf16x8 *>(reinterpret_cast<char *>(x_chunk(X, ldc, c, 0)) + (size_t)((uint32_t)r * 16u)) =
          frag8_zero();
  }
}

// The accepted block of parcel i: the predicted displacement, then the
// turbulent and mesoscale diffusion of the block's kSurrK steps with the
// random numbers the plain steps draw (Philox counters (id, step, 0) and
// (id, step, 1) for each step of the block) and the mesoscale spread of the
// cell holding the parcel at the block's start (at the first step's middle
// time); the summed displacement is converted to degrees and hPa at the
// displaced position, then one position fix.  lon, lat, p receive the final
// position.
__device__ __forceinline__ void apply_block(const StepArgs &a, int64_t i, double t0, float de, float dn,
                                            float dpp, float c0, double &lon, double &lat, double &p) {
  const float kdeg = (float)kDeg;
  const uint32_t id = a.id[i];
  float up = static_cast<const float *>(a.up)[i];
  float vp = static_cast<const float *>(a.vp)[i];
  float wp = static_cast<const float *>(a.wp)[i];
  const bool meso_on = (a.flags & kMeso) != 0;
  float sg[3] = {0.f, 0.f, 0.f};
  if (meso_on) {
    Loc<float> L0;
    surr_locate(a, lon, lat, p, t0 + 0.5 * a.dt, L0);
    const float4 x = reinterpret_cast<const float4 *>(a.sig)[(size_t)L0.l * (size_t)a.level_elems +
                                                             (size_t)((L0.k * a.ny + L0.j) * a.nx + L0.i0)];
    sg[0] = x.x; sg[1] = x.y; sg[2] = x.z;
  }
  lon = lon + (double)(de * 1000.0f * kdeg / c0);
  lat = lat + (double)(dn * 1000.0f * kdeg);
  p = p + (double)dpp;
  position(a, lon, lat, p);
  if (a.flags & (kTurb | kMeso)) {
    float ex = 0.f, ny = 0.f, dz = 0.f, dpm = 0.f;     // m east, m north, m up; hPa
    const float r = (float)a.r_ar, fdt = (float)a.dt;
    const float cu = (float)a.rs_fh * sg[0], cv = (float)a.rs_fh * sg[1], cw = (float)a.rs_fv * sg[2];
    for (int s = 0; s < kSurrK; ++s) {
      const uint32_t step = a.step0 + (uint32_t)s;
      if (a.flags & kTurb) {
        float xi[3];
        normals3<float>(a.seed, id, step, 0u, xi);
        ex += (float)a.sig_h * xi[0];
        ny += (float)a.sig_h * xi[1];
        dz += (float)a.sig_z * xi[2];
      }
      if (meso_on) {
        float xi[3];
        normals3<float>(a.seed, id, step, 1u, xi);
        up = fma(r, up, cu * xi[0]);
        vp = fma(r, vp, cv * xi[1]);
        wp = fma(r, wp, cw * xi[2]);
        ex += up * fdt;
        ny += vp * fdt;
        dpm += wp * fdt;
      }
    }
    const float c1 = cos_floor<float>(a, lat);
    lon = lon + (double)(ex * kdeg / c1);
    lat = lat + (double)(ny * kdeg);
    p = p + (double)(-dz * (float)p * (float)(1.0 / kH0) + dpm);
    position(a, lon, lat, p);
  }
  a.lon[i] = lon;
  a.lat[i] = lat;
  a.p[i] = p;
  static_cast<float *>(a.up)[i] = up;
  static_cast<float *>(a.vp)[i] = vp;
  static_cast<float *>(a.wp)[i] = wp;
}

// Consistency estimate, then acceptance (displacement, then the block's
// diffusion) or fallback, for parcels i0 .. i0 + cnt - 1 with predictions Y
// (4 floats per row).  Every wave
// records the ballot of its parcels that fall back in fb_mask[i / 64]
// (i0 is a multiple of 64), from which an ordered list is built.
__global__ __launch_bounds__(256) void k_surr_apply(const StepArgs a, float tau_km, const float *Y,
                                                    int64_t i0, int64_t cnt, float *err_out,
                                                    uint64_t *fb_mask) {
  const int lb = logical_block((int)blockIdx.x, a.per_xcd);
  if (lb >= a.nblk) return;
  const int64_t r = (int64_t)lb * 256 + threadIdx.x;
  const int l = threadIdx.x & 63;
  if (r - l >= cnt) return;                          // the whole wave is past the chunk
  const int64_t i = i0 + r;
  const bool in_range = r < cnt;
  double lon = 0.0, lat = 0.0, p = 0.0;
  if (in_range) {
    lon = a.lon[i];
    lat = a.lat[i];
    p = a.p[i];
  }
  const bool valid = in_range && finite3(lon, lat, p);
  const double t0 = a.t_start + (double)a.step0 * a.dt;
  const float kdeg = (float)kDeg;
  float de = 0.f, dn = 0.f, dpp = 0.f, c0 = 1.f;
  bool accept = false;
  if (valid) {
    const float4 yv = *reinterpret_cast<const float4 *>(Y + r * 4);
    de = yv.x;
    dn = yv.y;
    dpp = yv.z;
    // consistency estimate: kSurrK dt times the wind at the predicted midpoint
    c0 = cos_floor<float>(a, lat);
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
    accept = err <= tau_km && isfinite(err);
  }
  // parcels that fall back keep their state here; the plain step kernel
  // takes them from the ordered list (whose scan also gives their count)
  const uint64_t fb = __ballot(valid && !accept);
  if (l == 0) fb_mask[i / 64] = fb;
  if (valid && accept) apply_block(a, i, t0, de, dn, dpp, c0, lon, lat, p);
  if (a.sk) {
    // keys for the sort that follows: accepted parcels (final position) and
    // non-finite ones here, fallbacks after their plain steps
    const SortKeyArgs sk = *a.sk;
    const bool keyed = in_range && (accept || !valid);
    const uint32_t key = keyed ? tile_key(a, sk, a.plev, a.lut, lon, lat, p) : 0xFFFFFFFFu;
    const uint32_t rank = wave_key_rank(sk, key, keyed);
    if (keyed) {
      sk.keys[i] = key;
      sk.ranks[i] = rank;
    }
  }
}

// off[w] = number of set bits of fb_mask[w] for w < nw, off[nw] = 0.
__global__ void k_fb_counts(const uint64_t *fb_mask, int64_t nw, uint32_t *off) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w < nw) off[w] = (uint32_t)__popcll(fb_mask[w]);
  else if (w == nw) off[w] = 0u;
}

// After the exclusive scan of the counts: wave w's parcels that fall back
// go to list[off[w] ...] in increasing index order.
// Also adds the block's fallback count (the scan's total) to *fallbacks, from
// one thread: a per-wave atomic on that one counter serialized the apply
// kernel.
__global__ __launch_bounds__(256) void k_fb_expand(const uint64_t *fb_mask, int64_t nw, const uint32_t *off,
                                                   uint32_t *list, uint32_t *fallbacks) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *fallbacks += off[nw];
  const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (w >= nw) return;
  const int l = threadIdx.x & 63;
  const uint64_t m = fb_mask[w];
  if ((m >> l) & 1ull) list[off[w] + __popcll(m & ((1ull << l) - 1ull))] = (uint32_t)(w * 64 + l);
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

hipError_t launch_surr_pack_inf(const uint16_t *wt, uint16_t *wi, hipStream_t s) {
  hipLaunchKernelGGL(k_surr_pack_inf, dim3((kWiSize + 255) / 256), dim3(256), 0, s, wt, wi);
  return hipGetLastError();
}

hipError_t launch_surr_forward(const SurrW &W, const float *x, int64_t n, uint16_t *X, float *y,
                               int64_t chunk, hipStream_t s) {
  for (int64_t i0 = 0; i0 < n; i0 += chunk) {
    const int64_t cnt = n - i0 < chunk ? n - i0 : chunk;
    hipLaunchKernelGGL(k_surr_xnorm, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, W,
                       x + i0 * kSurrIn, cnt, X, chunk);
    const hipError_t e = launch_surr_mlp(W, X, cnt, chunk, y + i0 * kSurrOut, kSurrOut, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_surr_mlp(const SurrW &W, const uint16_t *X, int64_t n, int64_t ldc, float *Y, int ldy,
                           hipStream_t s) {
  const int64_t groups = (n + 63) / 64;
  const int64_t want = (groups + kMlpThreads / 64 - 1) / (kMlpThreads / 64);
  const unsigned nb = (unsigned)(want < kMlpBlocks ? want : kMlpBlocks);
  hipLaunchKernelGGL(k_surr_mlp, dim3(nb), dim3(kMlpThreads), 0, s, W, X, n, ldc, Y, ldy);
  return hipGetLastError();
}

// Per-chunk launch shape of the one-parcel-per-thread passes.
static StepArgs chunk_args(const StepArgs &a, int64_t cnt) {
  StepArgs c = a;
  const int64_t nblk = (cnt + 255) / 256;
  c.nblk = (int32_t)nblk;
  c.per_xcd = (int32_t)((nblk + kXcds - 1) / kXcds);
  return c;
}

hipError_t launch_surr_tfield(const StepArgs &a, double t, float4 *F, hipStream_t s) {
  hipLaunchKernelGGL(k_surr_tfield, dim3(4096), dim3(256), 0, s, a, t, F);
  return hipGetLastError();
}

hipError_t launch_surr_x(const StepArgs &a, const SurrW &W, const float4 *F, int64_t i0, int64_t cnt,
                         uint16_t *X, int64_t ldc, hipStream_t s) {
  if (cnt > ldc) return hipErrorInvalidValue;
  const StepArgs c = chunk_args(a, cnt);
  hipLaunchKernelGGL(k_surr_x, dim3((unsigned)(c.per_xcd * kXcds)), dim3(256), 0, s, c, W, F, i0, cnt, X, ldc);
  return hipGetLastError();
}

hipError_t launch_surr_apply(const StepArgs &a, float tau_km, const float *Y, int64_t i0, int64_t cnt,
                             float *err_out, uint64_t *fb_mask, hipStream_t s) {
  const StepArgs c = chunk_args(a, cnt);
  hipLaunchKernelGGL(k_surr_apply, dim3((unsigned)(c.per_xcd * kXcds)), dim3(256), 0, s, c, tau_km, Y, i0,
                     cnt, err_out, fb_mask);
  return hipGetLastError();
}

hipError_t launch_surr_fblist(const uint64_t *fb_mask, int64_t n, uint32_t *off, uint32_t *sums,
                              uint32_t *list, uint32_t *fallbacks, hipStream_t s) {
  const int64_t nw = (n + 63) / 64;
  hipLaunchKernelGGL(k_fb_counts, dim3((unsigned)((nw + 1 + 255) / 256)), dim3(256), 0, s, fb_mask, nw, off);
  const hipError_t e = launch_scan_u32(off, (uint32_t)(nw + 1), sums, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fb_expand, dim3((unsigned)((nw * 64 + 255) / 256)), dim3(256), 0, s, fb_mask, nw, off,
                     list, fallbacks);
  return hipGetLastError();
}

// Splits of the batch for the weight gradients: about 256 rows each, at
// most 16 (the 191 tiles x 16 shares fill the chip).
static hipError_t launch_wgrad(const SurrTrain &T, hipStream_t s) {
  int64_t split = T.batch / 256;
  if (split < 1) split = 1;
  if (split > 16) split = 16;
  const hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(T.grad), (uint32_t)kSurrNParam, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_surr_wgrad, dim3(48 + 64 + 64 + 8 + 7, (unsigned)split), dim3(64), 0, s, T, T.grad);
  return hipGetLastError();
}

hipError_t launch_surr_train(const SurrW &W, const SurrTrain &T, float *params, float *m, float *v,
                             float lr, float bc1, float bc2, hipStream_t s) {
  const unsigned nb = (unsigned)(T.batch / 64);
  hipLaunchKernelGGL(k_surr_train_fwd, dim3(nb), dim3(64), 0, s, W, T);
  hipLaunchKernelGGL(k_surr_train_bwd, dim3(nb), dim3(64), 0, s, W, T);
  if (launch_wgrad(T, s) != hipSuccess) return hipGetLastError();
  hipLaunchKernelGGL(k_surr_adam, dim3((kSurrNParam + 255) / 256), dim3(256), 0, s, params, T.grad, m, v,
                     lr, bc1, bc2);
  return hipGetLastError();
}

hipError_t launch_surr_grad(const SurrW &W, const SurrTrain &T, hipStream_t s) {
  const unsigned nb = (unsigned)(T.batch / 64);
  hipLaunchKernelGGL(k_surr_train_fwd, dim3(nb), dim3(64), 0, s, W, T);
  hipLaunchKernelGGL(k_surr_train_bwd, dim3(nb), dim3(64), 0, s, W, T);
  if (launch_wgrad(T, s) != hipSuccess) return hipGetLastError();
  return hipGetLastError();
}

}  // namespace mpt
