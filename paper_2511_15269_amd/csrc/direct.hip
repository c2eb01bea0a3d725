// Direct O(N * T) evaluation of the potential and field (eqs. 1-3): the
// reference against which the paper measures the FMM error (Sec. III.A).
// Thread = target; sources are staged through LDS in tiles of the block
// size.  Pairs at distance 0 contribute nothing.
#include "internal.h"

namespace fmm {
namespace {

constexpr double kInv4Pi = 0.079577471545947667884441881686257181;
constexpr int kTile = 256;

__device__ __forceinline__ double rsq(double r2) {
  double y = __builtin_amdgcn_rsq(r2);
  y = y * (1.5 - 0.5 * r2 * y * y);
  y = y * (1.5 - 0.5 * r2 * y * y);
  return y;
}
__device__ __forceinline__ float rsq(float r2) { return __builtin_amdgcn_rsqf(r2); }

template <typename T, bool FIELD>
__global__ __launch_bounds__(kTile) void k_direct(
    int64_t n, const double* __restrict__ pos, const T* __restrict__ q,
    const int64_t* __restrict__ targets, int64_t nt, T* __restrict__ pot,
    T* __restrict__ field) {
  __shared__ double sx[kTile], sy[kTile], sz[kTile];
  __shared__ T sq[kTile];
  const int64_t it = (int64_t)blockIdx.x * kTile + threadIdx.x;
  const bool live = it < nt;
  const int64_t t0 = live ? (targets ? targets[it] : it) : 0;
  const bool inside = t0 >= 0 && t0 < n;  // an index outside [0, n) reads nothing
  const int64_t ti = inside ? t0 : 0;
  const double xi = pos[3 * ti], yi = pos[3 * ti + 1], zi = pos[3 * ti + 2];
  T u = T(0), gx = T(0), gy = T(0), gz = T(0);
  for (int64_t base = 0; base < n; base += kTile) {
    const int64_t j = base + threadIdx.x;
    __syncthreads();
    if (j < n) {
      sx[threadIdx.x] = pos[3 * j];
      sy[threadIdx.x] = pos[3 * j + 1];
      sz[threadIdx.x] = pos[3 * j + 2];
      sq[threadIdx.x] = q[j];
    } else {
      sx[threadIdx.x] = xi;  // coincides with the target: contributes nothing
      sy[threadIdx.x] = yi;
      sz[threadIdx.x] = zi;
      sq[threadIdx.x] = T(0);
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < kTile; ++k) {
      const T dx = T(xi - sx[k]), dy = T(yi - sy[k]), dz = T(zi - sz[k]);
      const T r2 = dx * dx + dy * dy + dz * dz;
      const T inv = r2 > T(0) ? rsq(r2) : T(0);
      const T qi = sq[k] * inv;
      u += qi;
      if (FIELD) {
        const T q3 = qi * inv * inv;
        gx = fma(q3, dx, gx);
        gy = fma(q3, dy, gy);
        gz = fma(q3, dz, gz);
      }
    }
  }
  if (live) {
    const T bad = __builtin_nan("");
    pot[it] = inside ? -T(kInv4Pi) * u : bad;
    if (FIELD) {
      // field = -grad u = -(1/4pi) sum q (x_i - x_j)/r^3
      field[3 * it] = inside ? -T(kInv4Pi) * gx : bad;
      field[3 * it + 1] = inside ? -T(kInv4Pi) * gy : bad;
      field[3 * it + 2] = inside ? -T(kInv4Pi) * gz : bad;
    }
  }
}

template <typename T>
void launch(int64_t n, const double* pos, const void* q, const int64_t* targets,
            int64_t nt, void* pot, void* field, hipStream_t st) {
  const unsigned nb = (unsigned)((nt + kTile - 1) / kTile);
  if (field)
    k_direct<T, true><<<nb, kTile, 0, st>>>(n, pos, (const T*)q, targets, nt,
                                            (T*)pot, (T*)field);
  else
    k_direct<T, false><<<nb, kTile, 0, st>>>(n, pos, (const T*)q, targets, nt,
                                             (T*)pot, nullptr);
  FMM_HIP(hipGetLastError());
}

}  // namespace

void direct_sum(int64_t n, const double* pos, const void* q, int precision,
                const int64_t* targets, int64_t nt, void* pot, void* field,
                hipStream_t st) {
  if (nt == 0) return;
  if (precision == FMM_FP32)
    launch<float>(n, pos, q, targets, nt, pot, field, st);
  else
    launch<double>(n, pos, q, targets, nt, pot, field, st);
}

}  // namespace fmm
