// k_met.hip -- storing meteorological time levels in the kernel layout:
// one {u, v, w, T} record per grid point (T, the temperature, is 0 unless
// stored for convection / sedimentation), longitude fastest, so that a cell
// corner is one 16-byte (F32) or 8-byte (BF16 / F16) load.  Reduced
// precision stores q = RNE(f * (1/s)) with s = max|f| per (variable, level).
#include "mpt_internal.h"

namespace mpt {

__global__ __launch_bounds__(256) void k_pack_f32(const float *__restrict__ u,
                                                  const float *__restrict__ v,
                                                  const float *__restrict__ w,
                                                  float4 *__restrict__ dst, int64_t npts) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < npts; q += stride)
    dst[q] = make_float4(u[q], v[q], w[q], 0.0f);
}

// One block per (level k, variable): max |f| over the nx*ny points of that
// level; a zero maximum is stored as scale 1 (then every q is 0).
__global__ __launch_bounds__(256) void k_level_absmax(const float *__restrict__ u,
                                                      const float *__restrict__ v,
                                                      const float *__restrict__ w, int64_t nxy,
                                                      int nz, float *__restrict__ scales) {
  const int k = blockIdx.x, var = blockIdx.y;
  const float *src = (var == 0 ? u : var == 1 ? v : w) + (int64_t)k * nxy;
  float m = 0.0f;
  for (int64_t q = threadIdx.x; q < nxy; q += blockDim.x) m = fmaxf(m, fabsf(src[q]));
  __shared__ float red[256];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) scales[var * nz + k] = red[0] > 0.0f ? red[0] : 1.0f;
}

__device__ __forceinline__ unsigned short to_bf16_rne(float x) {
  uint32_t b = __float_as_uint(x);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (unsigned short)(b >> 16);
}

// The FP32 product is rounded first and only then converted: the empty asm
// pins x as a 32-bit register value, which keeps the compiler from fusing
// multiply and conversion into one mixed-precision FMA (a single rounding
// of the exact product instead of the defined FP32-then-FP16 rounding).
__device__ __forceinline__ unsigned short to_f16_rne(float x) {
  asm volatile("" : "+v"(x));
  return __builtin_bit_cast(unsigned short, (_Float16)x);
}

template <int F>
__global__ __launch_bounds__(256) void k_pack_r16(const float *__restrict__ u,
                                                  const float *__restrict__ v,
                                                  const float *__restrict__ w,
                                                  const float *__restrict__ scales,
                                                  ushort4 *__restrict__ dst, int64_t nxy, int nz) {
  const int64_t npts = nxy * nz;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < npts; q += stride) {
    const int k = (int)(q / nxy);
    const float iu = __fdiv_rn(1.0f, scales[k]);
    const float iv = __fdiv_rn(1.0f, scales[nz + k]);
    const float iw = __fdiv_rn(1.0f, scales[2 * nz + k]);
    const float a = __fmul_rn(u[q], iu), b = __fmul_rn(v[q], iv), c = __fmul_rn(w[q], iw);
    ushort4 r;
    if (F == kBF16) {
      r.x = to_bf16_rne(a); r.y = to_bf16_rne(b); r.z = to_bf16_rne(c);
    } else {
      r.x = to_f16_rne(a); r.y = to_f16_rne(b); r.z = to_f16_rne(c);
    }
    r.w = 0;
    dst[q] = r;
  }
}

// Temperature into the fourth value of each record of a stored level (the
// other three are left as they are).  F32: the float itself; R16: the code
// of T / s with the level's temperature scale s.
__global__ __launch_bounds__(256) void k_pack_temp_f32(const float *__restrict__ T,
                                                       float4 *__restrict__ dst, int64_t npts) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < npts; q += stride)
    reinterpret_cast<float *>(dst + q)[3] = T[q];
}

template <int F>
__global__ __launch_bounds__(256) void k_pack_temp_r16(const float *__restrict__ T,
                                                       const float *__restrict__ scales,
                                                       ushort4 *__restrict__ dst, int64_t nxy, int nz) {
  const int64_t npts = nxy * nz;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < npts; q += stride) {
    const int k = (int)(q / nxy);
    const float a = __fmul_rn(T[q], __fdiv_rn(1.0f, scales[k]));
    reinterpret_cast<unsigned short *>(dst + q)[3] = F == kBF16 ? to_bf16_rne(a) : to_f16_rne(a);
  }
}

// Surface records {cape, pel, ps, 0}.
__global__ __launch_bounds__(256) void k_pack_sfc(const float *__restrict__ cape,
                                                  const float *__restrict__ pel,
                                                  const float *__restrict__ ps,
                                                  float4 *__restrict__ dst, int64_t nxy) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nxy; q += stride)
    dst[q] = make_float4(cape[q], pel[q], ps[q], 0.0f);
}

// Spread table of one pair of time levels (ring slots s0 < earlier, s1):
// for every cell (k, j, i) with j < ny - 1 and k < nz - 1 the population
// standard deviation of each variable over the cell's 16 stored values (8
// corners x 2 levels; R16 decoded with the per-level scales), in FP64, two
// passes (mean, then squared deviations).  Cells of the last row and level
// are never read and get 0.  Stored {su, sv, sw, 0} as double (D) or float.
template <int F, bool D>
__global__ __launch_bounds__(256) void k_cell_sigma(const void *__restrict__ met, const float *__restrict__ scales,
                                                    int s0, int s1, int64_t level_elems, int nx, int ny, int nz,
                                                    void *__restrict__ out) {
  using T = typename Rec<F>::T;
  const int npts = nx * ny * nz;                     // < 2^31
  const int stride = (int)(gridDim.x * blockDim.x);
  for (int q = (int)(blockIdx.x * blockDim.x + threadIdx.x); q < npts; q += stride) {
    const int i = q % nx, r = q / nx;
    const int j = r % ny, k = r / ny;
    double sg[3] = {0.0, 0.0, 0.0};
    if (j < ny - 1 && k < nz - 1) {
      const int i1 = i + 1 == nx ? 0 : i + 1;
      double x[3][16];
      int n = 0;
#pragma unroll
      for (int dl = 0; dl < 2; ++dl) {
        const int slot = dl ? s1 : s0;
        const T *lev = reinterpret_cast<const T *>(met) + (size_t)slot * (size_t)level_elems;
#pragma unroll
        for (int dk = 0; dk < 2; ++dk)
#pragma unroll
          for (int dj = 0; dj < 2; ++dj)
#pragma unroll
            for (int di = 0; di < 2; ++di) {
              const T v = lev[((k + dk) * ny + j + dj) * nx + (di ? i1 : i)];
              if constexpr (F == kF32) {
                x[0][n] = (double)v.x;
                x[1][n] = (double)v.y;
                x[2][n] = (double)v.z;
              } else {
                const float *sc = scales + (size_t)slot * 3 * nz + (k + dk);
                x[0][n] = (double)(dec<F>(v.x) * sc[0]);
                x[1][n] = (double)(dec<F>(v.y) * sc[nz]);
                x[2][n] = (double)(dec<F>(v.z) * sc[2 * nz]);
              }
              ++n;
            }
      }
#pragma unroll
      for (int var = 0; var < 3; ++var) {
        double mean = 0.0;
#pragma unroll
        for (int m = 0; m < 16; ++m) mean += x[var][m];
        mean /= 16.0;
        double ss = 0.0;
#pragma unroll
        for (int m = 0; m < 16; ++m) ss += (x[var][m] - mean) * (x[var][m] - mean);
        ss /= 16.0;
        sg[var] = sqrt(ss > 0.0 ? ss : 0.0);
      }
    }
    if constexpr (D) {
      double2 *o = static_cast<double2 *>(out) + 2 * (size_t)q;
      o[0] = make_double2(sg[0], sg[1]);
      o[1] = make_double2(sg[2], 0.0);
    } else {
      static_cast<float4 *>(out)[q] = make_float4((float)sg[0], (float)sg[1], (float)sg[2], 0.0f);
    }
  }
}

__global__ __launch_bounds__(256) void k_fill_f32(float *dst, float value, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) dst[q] = value;
}

static unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

hipError_t launch_pack_f32(const float *u, const float *v, const float *w, float4 *dst, int64_t npts,
                           hipStream_t stream) {
  hipLaunchKernelGGL(k_pack_f32, dim3(grid_for(npts)), dim3(256), 0, stream, u, v, w, dst, npts);
  return hipGetLastError();
}

hipError_t launch_level_absmax(const float *u, const float *v, const float *w, int64_t nxy, int nz,
                               float *scales, hipStream_t stream) {
  hipLaunchKernelGGL(k_level_absmax, dim3((unsigned)nz, 3), dim3(256), 0, stream, u, v, w, nxy, nz,
                     scales);
  return hipGetLastError();
}

hipError_t launch_pack_r16(int field, const float *u, const float *v, const float *w,
                           const float *scales, ushort4 *dst, int64_t nxy, int nz,
                           hipStream_t stream) {
  const unsigned g = grid_for(nxy * nz);
  if (field == kBF16)
    hipLaunchKernelGGL(k_pack_r16<kBF16>, dim3(g), dim3(256), 0, stream, u, v, w, scales, dst, nxy, nz);
  else
    hipLaunchKernelGGL(k_pack_r16<kF16>, dim3(g), dim3(256), 0, stream, u, v, w, scales, dst, nxy, nz);
  return hipGetLastError();
}

hipError_t launch_pack_temp(int field, const float *T, float *t_scales, void *dst, int64_t nxy, int nz,
                            hipStream_t stream) {
  const unsigned g = grid_for(nxy * nz);
  if (field == kF32) {
    hipLaunchKernelGGL(k_pack_temp_f32, dim3(g), dim3(256), 0, stream, T, static_cast<float4 *>(dst),
                       nxy * nz);
    return hipGetLastError();
  }
  // one block per level: max |T| into t_scales[k] (the u slot of the kernel)
  hipLaunchKernelGGL(k_level_absmax, dim3((unsigned)nz, 1), dim3(256), 0, stream, T, T, T, nxy, nz,
                     t_scales);
  if (field == kBF16)
    hipLaunchKernelGGL(k_pack_temp_r16<kBF16>, dim3(g), dim3(256), 0, stream, T, t_scales,
                       static_cast<ushort4 *>(dst), nxy, nz);
  else
    hipLaunchKernelGGL(k_pack_temp_r16<kF16>, dim3(g), dim3(256), 0, stream, T, t_scales,
                       static_cast<ushort4 *>(dst), nxy, nz);
  return hipGetLastError();
}

hipError_t launch_pack_sfc(const float *cape, const float *pel, const float *ps, float4 *dst, int64_t nxy,
                           hipStream_t stream) {
  hipLaunchKernelGGL(k_pack_sfc, dim3(grid_for(nxy)), dim3(256), 0, stream, cape, pel, ps, dst, nxy);
  return hipGetLastError();
}

hipError_t launch_cell_sigma(int field, bool f64, const void *met, const float *scales, int s0, int s1,
                             int64_t level_elems, int nx, int ny, int nz, void *out, hipStream_t stream) {
  const dim3 g(grid_for(level_elems)), b(256);
  if (field == kF32) {
    if (f64) hipLaunchKernelGGL((k_cell_sigma<kF32, true>), g, b, 0, stream, met, scales, s0, s1, level_elems, nx, ny, nz, out);
    else hipLaunchKernelGGL((k_cell_sigma<kF32, false>), g, b, 0, stream, met, scales, s0, s1, level_elems, nx, ny, nz, out);
  } else if (field == kBF16) {
    hipLaunchKernelGGL((k_cell_sigma<kBF16, false>), g, b, 0, stream, met, scales, s0, s1, level_elems, nx, ny, nz, out);
  } else {
    hipLaunchKernelGGL((k_cell_sigma<kF16, false>), g, b, 0, stream, met, scales, s0, s1, level_elems, nx, ny, nz, out);
  }
  return hipGetLastError();
}

hipError_t launch_fill_f32(float *dst, float value, int64_t n, hipStream_t stream) {
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n)), dim3(256), 0, stream, dst, value, n);
  return hipGetLastError();
}

}  // namespace mpt
