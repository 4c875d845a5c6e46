// Processing steps around the RPCA solve, on the device (rpca_frame_* /
// rpca_moving_average / rpca_dice / rpca_rmse / rpca_masked_mean in
// include/rpca.h):
//
//   * consecutive-frame correlation, used to drop frames that correlate
//     poorly with their neighbours (the paper's in vivo reference, Sec. III);
//   * frame selection (copy of the kept frames into a new Casorati matrix);
//   * temporal moving average over W frames (same passage);
//   * binarisation and the Dice coefficient (Sec. II-F, Eq. 8), the RMSE
//     (Eq. 7) and the masked mean that gives the binarisation threshold.
//
// Every reduction is fixed-order: each workgroup writes a partial to its own
// slot and one more launch adds the slots in order, so results do not
// depend on scheduling.  Sums are FP64, counts are 64-bit integers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "rpca.h"
#include "common.h"
#include "engine.h"

namespace rpca {
namespace {

constexpr int kPT = 256;        // threads per workgroup
constexpr int kMaxGrid = 1024;  // workgroups of a reduction pass
constexpr int kCorrMaxN = 160;  // frames handled by the correlation kernel

__device__ inline double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ inline long long wsum_i(long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sums of frame t, its square and its product with frame t+1 over one run
// of rows: workgroup (rb, t) writes partial[rb][3t .. 3t+2].  Each thread
// accumulates over its rows in registers; one workgroup reduction at the end.
template <typename T>
__global__ void __launch_bounds__(kPT)
k_frame_sums(const T* __restrict__ X, int64_t m, int n, double* __restrict__ partial) {
  __shared__ double red[kPT / 64][3];
  const int t = blockIdx.y;
  const int64_t per = (m + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = blockIdx.x * per, r1 = r0 + per < m ? r0 + per : m;
  const T* xt = X + static_cast<size_t>(t) * m;
  const T* xn = X + static_cast<size_t>(t + 1 < n ? t + 1 : t) * m;
  double s = 0.0, q = 0.0, c = 0.0;
  for (int64_t p = r0 + threadIdx.x; p < r1; p += kPT) {
    const double x = static_cast<double>(xt[p]);
    s += x;
    q = fma(x, x, q);
    if (t + 1 < n) c = fma(x, static_cast<double>(xn[p]), c);
  }
  s = wsum(s);
  q = wsum(q);
  c = wsum(c);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[wv][0] = s;
    red[wv][1] = q;
    red[wv][2] = c;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double v = red[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < kPT / 64; ++w) v += red[w][threadIdx.x];
    partial[static_cast<size_t>(blockIdx.x) * 3 * n + 3 * t + threadIdx.x] = v;
  }
}

// Sum `slots` partials of `len` doubles in slot order into out[len].
__global__ void __launch_bounds__(kPT)
k_sum_slots(const double* __restrict__ partial, int slots, int len, double* __restrict__ out) {
  for (int i = threadIdx.x; i < len; i += kPT) {
    double v = 0.0;
    for (int s = 0; s < slots; ++s) v += partial[static_cast<size_t>(s) * len + i];
    out[i] = v;
  }
}

__global__ void __launch_bounds__(kPT)
k_sum_slots_i(const long long* __restrict__ partial, int slots, int len, long long* __restrict__ out) {
  for (int i = threadIdx.x; i < len; i += kPT) {
    long long v = 0;
    for (int s = 0; s < slots; ++s) v += partial[static_cast<size_t>(s) * len + i];
    out[i] = v;
  }
}

// out[:, t] = mean of M[:, t .. t+W-1], t = 0 .. n-W.  One thread per pixel
// row keeps the last W values in an LDS ring and a running FP64 sum, so each
// input is read once and each output written once.
constexpr int kMAT = 128;  // threads of the moving-average kernel (LDS ring W x 128)

template <typename T>
__global__ void __launch_bounds__(kMAT)
k_moving_average(const T* __restrict__ X, int64_t m, int n, int W, T* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char ring_raw[];
  T* ring = reinterpret_cast<T*>(ring_raw);
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kMAT + threadIdx.x;
  if (p >= m) return;
  const double inv = 1.0 / static_cast<double>(W);
  double sum = 0.0;
  for (int t = 0; t < n; ++t) {
    const T x = X[static_cast<size_t>(t) * m + p];
    T* slot = ring + static_cast<size_t>(t % W) * kMAT + threadIdx.x;
    if (t >= W) sum -= static_cast<double>(*slot);
    *slot = x;
    sum += static_cast<double>(x);
    if (t >= W - 1) out[static_cast<size_t>(t - W + 1) * m + p] = static_cast<T>(sum * inv);
  }
}

// counts[slot][3] = |A >= ta & B >= tb|, |A >= ta|, |B >= tb| (compared in FP64)
template <typename T>
__global__ void __launch_bounds__(kPT)
k_dice_counts(const T* __restrict__ A, double ta, const T* __restrict__ B, double tb, int64_t count,
              long long* __restrict__ partial) {
  __shared__ long long red[kPT / 64][3];
  long long both = 0, ca = 0, cb = 0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kPT) + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * kPT) {
    const bool a = static_cast<double>(A[i]) >= ta, b = static_cast<double>(B[i]) >= tb;
    both += (a && b) ? 1 : 0;
    ca += a ? 1 : 0;
    cb += b ? 1 : 0;
  }
  both = wsum_i(both);
  ca = wsum_i(ca);
  cb = wsum_i(cb);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[wv][0] = both;
    red[wv][1] = ca;
    red[wv][2] = cb;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    long long v = 0;
    for (int w = 0; w < kPT / 64; ++w) v += red[w][threadIdx.x];
    partial[static_cast<size_t>(blockIdx.x) * 3 + threadIdx.x] = v;
  }
}

// partial[slot][2] = sum over the slot of (A - B)^2 and of 1 (MODE 0), or of
// A * [mask != 0] and [mask != 0] (MODE 1).
template <typename T, int MODE>
__global__ void __launch_bounds__(kPT)
k_pair_sums(const T* __restrict__ A, const void* __restrict__ Bv, int64_t count,
            double* __restrict__ partial) {
  __shared__ double red[kPT / 64][2];
  double s = 0.0, c = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kPT) + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * kPT) {
    const double a = static_cast<double>(A[i]);
    if constexpr (MODE == 0) {
      const double dlt = a - static_cast<double>(static_cast<const T*>(Bv)[i]);
      s = fma(dlt, dlt, s);
      c += 1.0;
    } else {
      const bool on = static_cast<const uint8_t*>(Bv)[i] != 0;
      s += on ? a : 0.0;
      c += on ? 1.0 : 0.0;
    }
  }
  s = wsum(s);
  c = wsum(c);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[wv][0] = s;
    red[wv][1] = c;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double v = red[0][threadIdx.x];
    for (int w = 1; w < kPT / 64; ++w) v += red[w][threadIdx.x];
    partial[static_cast<size_t>(blockIdx.x) * 2 + threadIdx.x] = v;
  }
}

int grid_for(int64_t count) {
  const int64_t g = (count + kPT * 8 - 1) / (kPT * 8);
  return static_cast<int>(g < 1 ? 1 : (g > kMaxGrid ? kMaxGrid : g));
}

// Run a partial-producing launch, sum its slots in order and copy `len`
// results to host memory `out` (stream-ordered, then synchronised).
template <typename V, typename Launch, typename SumKernel>
int reduce_to_host(hipStream_t s, int grid, int len, V* out, Launch&& launch, SumKernel sumk) {
  V* buf = nullptr;
  const size_t bytes = sizeof(V) * (static_cast<size_t>(grid) + 1) * len;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&buf), bytes, s);
  if (e != hipSuccess || !buf) {
    set_error("hipMallocAsync(reduction)", e);
    (void)hipGetLastError();
    return RPCA_ERR_NOMEM;
  }
  V* total = buf + static_cast<size_t>(grid) * len;
  launch(buf);
  e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(sumk, dim3(1), dim3(kPT), 0, s, buf, grid, len, total);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out, total, sizeof(V) * len, hipMemcpyDeviceToHost, s);
  const hipError_t ef = hipFreeAsync(buf, s);
  if (e == hipSuccess) e = ef;
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    set_error("reduction", e);
    return RPCA_ERR_DEVICE;
  }
  return RPCA_OK;
}

bool dtype_ok(int32_t dtype) { return dtype == RPCA_F32 || dtype == RPCA_F64; }

}  // namespace
}  // namespace rpca

using namespace rpca;

extern "C" {

int rpca_frame_correlation(const void* M, int64_t m, int64_t n, int32_t dtype, double* rho,
                           void* stream) {
  if (!M || !rho || m < 2 || n < 2 || n > kCorrMaxN || !dtype_ok(dtype)) return RPCA_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // row blocks per frame: enough workgroups in total to fill the device
  const int64_t rbs = (m + 16 * kPT - 1) / (16 * kPT);
  const int grid = static_cast<int>(rbs < 1 ? 1 : (rbs > 64 ? 64 : rbs));
  const int len = static_cast<int>(3 * n);
  std::vector<double> sums(len);
  const int rc = reduce_to_host(s, grid, len, sums.data(), [&](double* buf) {
    const dim3 g(grid, static_cast<unsigned>(n));
    if (dtype == RPCA_F32)
      hipLaunchKernelGGL(k_frame_sums<float>, g, dim3(kPT), 0, s, static_cast<const float*>(M), m,
                         static_cast<int>(n), buf);
    else
      hipLaunchKernelGGL(k_frame_sums<double>, g, dim3(kPT), 0, s, static_cast<const double*>(M), m,
                         static_cast<int>(n), buf);
  }, k_sum_slots);
  if (rc != RPCA_OK) return rc;
  const double mm = static_cast<double>(m);
  for (int64_t t = 0; t + 1 < n; ++t) {
    const double sx = sums[3 * t], sxx = sums[3 * t + 1], sxy = sums[3 * t + 2];
    const double sy = sums[3 * (t + 1)], syy = sums[3 * (t + 1) + 1];
    const double cov = sxy - sx * sy / mm;
    const double vx = sxx - sx * sx / mm, vy = syy - sy * sy / mm;
    rho[t] = (vx > 0.0 && vy > 0.0) ? cov / std::sqrt(vx * vy) : 0.0;
  }
  return RPCA_OK;
}

int rpca_frame_keep(const double* rho, int64_t n, double threshold, int32_t* keep) {
  if (!rho || !keep || n < 1) return RPCA_ERR_ARG;
  int kept = 0;
  for (int64_t t = 0; t < n; ++t) {
    double best = -2.0;
    if (t > 0) best = std::fmax(best, rho[t - 1]);
    if (t + 1 < n) best = std::fmax(best, rho[t]);
    keep[t] = (n == 1 || best >= threshold) ? 1 : 0;
    kept += keep[t];
  }
  return kept;
}

int rpca_frame_select(const void* M, int64_t m, int64_t n, int32_t dtype, const int32_t* keep,
                      void* out, void* stream) {
  if (!M || !out || !keep || m < 1 || n < 1 || !dtype_ok(dtype)) return RPCA_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t col = static_cast<size_t>(m) * (dtype == RPCA_F32 ? 4 : 8);
  int k = 0;
  for (int64_t t = 0; t < n; ++t) {
    if (!keep[t]) continue;
    const hipError_t e = hipMemcpyAsync(static_cast<char*>(out) + col * k,
                                        static_cast<const char*>(M) + col * t, col,
                                        hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) {
      set_error("hipMemcpyAsync(frame)", e);
      return RPCA_ERR_DEVICE;
    }
    ++k;
  }
  return k;
}

int rpca_moving_average(const void* M, int64_t m, int64_t n, int32_t W, int32_t dtype, void* out,
                        void* stream) {
  if (!M || !out || m < 1 || W < 1 || W > 32 || n < W || !dtype_ok(dtype)) return RPCA_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int grid = static_cast<int>((m + kMAT - 1) / kMAT);
  const size_t lds = static_cast<size_t>(W) * kMAT * (dtype == RPCA_F32 ? 4 : 8);
  if (dtype == RPCA_F32)
    hipLaunchKernelGGL(k_moving_average<float>, dim3(grid), dim3(kMAT), lds, s,
                       static_cast<const float*>(M), m, static_cast<int>(n), W, static_cast<float*>(out));
  else
    hipLaunchKernelGGL(k_moving_average<double>, dim3(grid), dim3(kMAT), lds, s,
                       static_cast<const double*>(M), m, static_cast<int>(n), W, static_cast<double*>(out));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("k_moving_average", e);
    return RPCA_ERR_DEVICE;
  }
  return RPCA_OK;
}

int rpca_dice(const void* A, double thr_a, const void* B, double thr_b, int64_t count, int32_t dtype,
              int64_t* counts, double* dice, void* stream) {
  if (!A || !B || count < 1 || !dtype_ok(dtype)) return RPCA_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int grid = grid_for(count);
  long long c[3] = {0, 0, 0};
  const int rc = reduce_to_host(s, grid, 3, c, [&](long long* buf) {
    if (dtype == RPCA_F32)
      hipLaunchKernelGGL(k_dice_counts<float>, dim3(grid), dim3(kPT), 0, s, static_cast<const float*>(A),
                         thr_a, static_cast<const float*>(B), thr_b, count, buf);
    else
      hipLaunchKernelGGL(k_dice_counts<double>, dim3(grid), dim3(kPT), 0, s,
                         static_cast<const double*>(A), thr_a, static_cast<const double*>(B), thr_b,
                         count, buf);
  }, k_sum_slots_i);
  if (rc != RPCA_OK) return rc;
  if (counts)
    for (int i = 0; i < 3; ++i) counts[i] = c[i];
  if (dice) {
    const long long den = c[1] + c[2];
    *dice = den == 0 ? 1.0 : 2.0 * static_cast<double>(c[0]) / static_cast<double>(den);
  }
  return RPCA_OK;
}

int rpca_rmse(const void* A, const void* B, int64_t count, int32_t dtype, double* out, void* stream) {
  if (!A || !B || !out || count < 1 || !dtype_ok(dtype)) return RPCA_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int grid = grid_for(count);
  double r[2] = {0, 0};
  const int rc = reduce_to_host(s, grid, 2, r, [&](double* buf) {
    if (dtype == RPCA_F32)
      hipLaunchKernelGGL((k_pair_sums<float, 0>), dim3(grid), dim3(kPT), 0, s, static_cast<const float*>(A),
                         B, count, buf);
    else
      hipLaunchKernelGGL((k_pair_sums<double, 0>), dim3(grid), dim3(kPT), 0, s,
                         static_cast<const double*>(A), B, count, buf);
  }, k_sum_slots);
  if (rc != RPCA_OK) return rc;
  *out = std::sqrt(r[0] / static_cast<double>(count));
  return RPCA_OK;
}

int rpca_masked_mean(const void* A, const uint8_t* mask, int64_t count, int32_t dtype, double* out,
                     void* stream) {
  if (!A || !mask || !out || count < 1 || !dtype_ok(dtype)) return RPCA_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int grid = grid_for(count);
  double r[2] = {0, 0};
  const int rc = reduce_to_host(s, grid, 2, r, [&](double* buf) {
    if (dtype == RPCA_F32)
      hipLaunchKernelGGL((k_pair_sums<float, 1>), dim3(grid), dim3(kPT), 0, s, static_cast<const float*>(A),
                         mask, count, buf);
    else
      hipLaunchKernelGGL((k_pair_sums<double, 1>), dim3(grid), dim3(kPT), 0, s,
                         static_cast<const double*>(A), mask, count, buf);
  }, k_sum_slots);
  if (rc != RPCA_OK) return rc;
  *out = r[1] > 0.0 ? r[0] / r[1] : std::nan("");
  return r[1] > 0.0 ? RPCA_OK : RPCA_ERR_ARG;
}

}  // extern "C"
