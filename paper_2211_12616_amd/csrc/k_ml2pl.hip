// k_ml2pl.hip -- meteorological fields on hybrid model levels to the
// context's fixed pressure levels (the vertical regridding read_met does
// before the data are used, Sec. 3.1).  Column pressures p_k = a_k + b_k ps
// (decreasing with k); each target level p is interpolated linearly in ln p
// between the model levels bracketing it in its column; a target below the
// lowest or above the highest model level takes that level's value.
#include "mpt_device.h"
#include "mpt_internal.h"

namespace mpt {

// One thread per target point (m, j, i), longitude fastest.
__global__ __launch_bounds__(256) void k_ml_to_pl(const Ml2PlArgs g, const float *ps, const float *u,
                                                  const float *v, const float *w, float *uo, float *vo,
                                                  float *wo) {
  const int64_t ncol = (int64_t)g.nx * g.ny;
  const int64_t total = ncol * g.nz;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t col = q % ncol;
    const int m = (int)(q / ncol);
    const double s = (double)ps[col];
    const double pt = g.plev[m];
    const double *A = g.a, *B = g.b;
    int k0, k1;
    double wgt;
    if (pt >= A[0] + B[0] * s) {                 // at or below the lowest model level
      k0 = k1 = 0;
      wgt = 0.0;
    } else if (pt <= A[g.nml - 1] + B[g.nml - 1] * s) {   // at or above the highest
      k0 = k1 = g.nml - 1;
      wgt = 0.0;
    } else {
      int lo = 0, hi = g.nml - 2;                 // largest k with p_k >= pt
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (A[mid] + B[mid] * s >= pt) lo = mid; else hi = mid - 1;
      }
      k0 = lo;
      k1 = lo + 1;
      const double l0 = log(A[k0] + B[k0] * s), l1 = log(A[k1] + B[k1] * s);
      wgt = (l0 - log(pt)) / (l0 - l1);
    }
    const int64_t i0 = (int64_t)k0 * ncol + col, i1 = (int64_t)k1 * ncol + col;
    uo[q] = (float)((double)u[i0] + wgt * ((double)u[i1] - (double)u[i0]));
    vo[q] = (float)((double)v[i0] + wgt * ((double)v[i1] - (double)v[i0]));
    wo[q] = (float)((double)w[i0] + wgt * ((double)w[i1] - (double)w[i0]));
  }
}

hipError_t launch_ml_to_pl(const Ml2PlArgs &g, const float *ps, const float *u, const float *v,
                           const float *w, float *uo, float *vo, float *wo, hipStream_t s) {
  const int64_t total = (int64_t)g.nx * g.ny * g.nz;
  int64_t nb = (total + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_ml_to_pl, dim3((unsigned)nb), dim3(256), 0, s, g, ps, u, v, w, uo, vo, wo);
  return hipGetLastError();
}

}  // namespace mpt
