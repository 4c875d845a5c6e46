// Streaming kernels of the RPCA iteration (paper Sec. II-A, Eqs. 4-6).
//
// One thread owns one pixel row p of the Casorati matrix and holds its n
// frame values in registers (n <= NB, NB a compile-time frame class).  Frame
// j of row p sits at p + j*m, so for every j a wavefront reads 64 consecutive
// pixels: each load instruction is one coalesced 256 B (FP32) / 512 B (FP64)
// segment.  A workgroup processes one tile of kTile rows.
//
// k_stream<MODE=init>   : one pass over X.  sum|X|, sum X^2, non-finite count
//                         (for mu and the stopping test) and the Gram X^T X,
//                         which is the Gram of the first iterate because S and
//                         Y start at zero.
// k_stream<MODE=warm>   : for a solve started from S0, Y0: the Gram of
//                         A_1 = X - S0 + Y0/mu, copying S0 and Y0 into the
//                         buffers the first update pass reads.
// k_stream<MODE=update> : one ALM iteration k for every row, fused:
//                           a  = x - s + y/mu                  (argument of Eq. 4)
//                           l  = a P      P = V diag(w) V^T  (Eq. 4 rebuild)
//                           t  = x - l + y/mu
//                           s' = shrink_{lam/mu}(t)           (Eq. 5)
//                           z  = x - l - s'
//                           y' = y + mu z                      (Eq. 6)
//                           r2 += z^2                          (stopping test)
//                           a' = x - s' + y'/mu  -> Gram of the next iterate
//                         reading X, S_{k-1}, Y_{k-1} and writing S_k, Y_k:
//                         five words per matrix entry and iteration.
// k_finalize            : L = A_k P_k for the last iterate (same arithmetic as
//                         the rebuild above) and S_k, into the caller's buffers.
//
// Reductions never use floating-point atomics, and the streaming kernels use
// no cross-workgroup synchronisation at all: each workgroup writes its partial
// sums to a fixed slot; the next launch (k_reduce_groups) adds each group of
// kGroup slots in slot order, and the eigensolve kernel adds the group sums in
// group order.  Kernel boundaries order the steps.  The result depends only on
// the solve's own shape, so it is bitwise the same alone or in a batch.
#pragma once

#include "common.h"

namespace rpca {

__device__ inline void blk_coords(int blk, int& bi, int& bj) {
  int j = 0;
  while ((j + 1) * (j + 2) / 2 <= blk) ++j;
  bj = j;
  bi = blk - j * (j + 1) / 2;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// The value held by the partner lane in an aligned quad of lanes, for a DPP
// quad permutation CTRL.  Every lane of the wave must be active.
constexpr int kQuadXor1 = 0xB1;  // lanes [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;  // lanes [2,3,0,1]
template <int CTRL>
__device__ inline double quad_swap(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<unsigned>(b)), CTRL,
                                             0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<unsigned>(b >> 32)),
                                             CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, (static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
                                        static_cast<unsigned>(lo));
}

// Row chunks per 4x4 Gram block for nblk blocks: as many as the workgroup's
// threads give (at most 64), lowered to a multiple of 4 (else of 2) where
// that leaves the longest per-thread row loop as it is, so that aligned lane
// quads (pairs) can add their block sums in registers.
__host__ __device__ inline constexpr int gram_chunks(int nblk) {
  int c = kThreads / nblk;
  if (c > 64) c = 64;
  const int rows = (kTile + c - 1) / c;
  const int c4 = c & ~3, c2 = c & ~1;
  if (c4 > 0 && (kTile + c4 - 1) / c4 == rows) return c4;
  if (c2 > 0 && (kTile + c2 - 1) / c2 == rows) return c2;
  return c;
}
__host__ __device__ inline constexpr int gram_lane_group(int c) {
  return (c & 3) == 0 ? 4 : (c & 1) == 0 ? 2 : 1;
}
// LDS stride of one lane-group sum (16 doubles): 144 B keeps each entry
// 16 B aligned for b128 writes and puts the entries of consecutive writer
// lanes on different LDS banks.
constexpr int kRedLd = 18;
// LDS doubles that the lane-group sums of any frame count up to nb take.
constexpr int gram_red_doubles(int nb) {
  int most = 0;
  for (int n = 1; n <= nb; ++n) {
    const int nblk = gram_blocks((n + 3) >> 2);
    const int c = gram_chunks(nblk);
    const int need = nblk * (c / gram_lane_group(c)) * kRedLd;
    if (need > most) most = need;
  }
  return most;
}

// A value the compiler must treat as unknown at this point (an empty asm that
// claims to change it).  Applied per tile to the matrix base addresses and
// sizes in the loops over tiles, so that the per-frame column addresses are
// formed next to their use instead of being hoisted out of the loop and kept
// live across it (NB columns of five matrices would not fit the scalar
// registers).
template <typename V>
__device__ inline V opaque(V v) {
  static_assert(sizeof(V) == 8, "64-bit values");
  uint64_t u = __builtin_bit_cast(uint64_t, v);
  // the values are uniform over the workgroup: keep them in scalar registers
  uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u));
  uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u >> 32));
  asm volatile("" : "+s"(lo), "+s"(hi));
  return __builtin_bit_cast(V, (static_cast<uint64_t>(hi) << 32) | lo);
}

__device__ inline float clamp_sym(float v, float g) { return fminf(fmaxf(v, -g), g); }
__device__ inline double clamp_sym(double v, double g) { return fmin(fmax(v, -g), g); }
__device__ inline bool finite_val(float v) { return __builtin_isfinite(v); }
__device__ inline bool finite_val(double v) { return __builtin_isfinite(v); }

// MT: the work item may span several tiles (the solve's tiles per work item,
// d.tps).  The single-tile kernels (MT = false) keep their registers free of
// the Gram accumulators during the loads and the rebuild, which decides
// their occupancy; the loop costs about 40 registers.
template <typename T, int NB, int MODE, bool MT>
__global__ void __launch_bounds__(kThreads)
k_stream(const SolveDesc* __restrict__ descs, const WorkItem* __restrict__ items) {
  constexpr bool INIT = MODE == 0;  // kModeInit
  constexpr bool WARM = MODE == 3;  // kModeWarm
  constexpr int NB4 = (NB + 3) / 4 * 4;
  constexpr int LDT = kTile + 1;  // odd row stride: frames of one row fall in different banks
  constexpr size_t kTileBytes = sizeof(T) * NB4 * LDT;
  constexpr size_t kRedBytes = sizeof(double) * gram_red_doubles(NB);
  constexpr size_t kSmem = kTileBytes > kRedBytes ? kTileBytes : kRedBytes;
  __shared__ __align__(16) unsigned char smem[kSmem];
  __shared__ double wred[kThreads / 64][kScalars];
  T* tileA = reinterpret_cast<T*>(smem);
  double* red = reinterpret_cast<double*>(smem);

  const int tid = threadIdx.x;
  const int64_t t_begin = RPCA_NOW();
  const WorkItem wi = items[blockIdx.x];
  const SolveDesc& d = descs[wi.solve];
  SolveState* st = d.st;
  int k = 0;
  if constexpr (WARM) {
    if (st->done || st->warm_stage != 1) return;
  } else if constexpr (!INIT) {
    if (st->done) return;
    k = st->iter;
  }
  const int n = d.n;
  const int64_t m = d.m;
  const gptr<const T> X = as_global<T>(d.X);
  const gptr<const T> Sin = as_global<T>(static_cast<const void*>(d.S[(k + 1) & 1]));
  const gptr<const T> Yin = as_global<T>(static_cast<const void*>(d.Y[(k + 1) & 1]));
  const gptr<T> Sout = as_global<T>(d.S[k & 1]);
  const gptr<T> Yout = as_global<T>(d.Y[k & 1]);
  // S_0 = Y_0 = 0 are not read unless the solve starts from a given S0 / Y0
  const bool first = (k == 1) && !d.warm;
  T mu = 0, imu = 0, gam = 0;
  if constexpr (!INIT) {
    mu = static_cast<T>(st->mu);
    imu = static_cast<T>(st->imu);
    gam = static_cast<T>(st->gamma);
  }

  // Gram work split: 4x4 blocks of frames x C row chunks; aligned groups of
  // G lanes (chunks of one block) add in registers, leaving Q sums per block.
  const int nblk = gram_blocks((n + 3) >> 2);
  const int C = gram_chunks(nblk);
  const int G = gram_lane_group(C);
  const int Q = C / G;
  const int gblk = tid / C;
  const int gc = tid - gblk * C;
  const bool gact = gblk < nblk;
  int bi = 0, bj = 0;
  if (gact) blk_coords(gblk, bi, bj);
  double gacc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) gacc[e] = 0.0;
  double r2 = 0.0, s1 = 0.0, s2 = 0.0, nf = 0.0;

  // The work item's run of tiles: tiles [t0, t1) of kTile rows, walked in
  // order; the Gram accumulators and scalars run over all of them, so the
  // workgroup writes one partial.  Row index p within the solve (m < 2^30,
  // so byte offsets fit 32 bits).
  const int t0 = wi.slot * d.tps;
  const int t1 = MT ? min(t0 + d.tps, d.tiles) : t0 + 1;
  // Gram of the LDS tile (rows of this tile, A' frame-major), accumulated
  // into this thread's 4x4 block over its row chunk.
  auto gram_tile = [&]() {
    __syncthreads();
    if (gact) {
      const T* u = tileA + (4 * bi) * LDT;
      const T* v = tileA + (4 * bj) * LDT;
      for (int r = gc; r < kTile; r += C) {
        double ue[4], vf[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          ue[e] = static_cast<double>(u[e * LDT + r]);
          vf[e] = static_cast<double>(v[e * LDT + r]);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int f = 0; f < 4; ++f) gacc[e * 4 + f] = fma(ue[e], vf[f], gacc[e * 4 + f]);
      }
    }
    __syncthreads();
  };
  if constexpr (INIT) {
#pragma unroll 1
    for (int tile = t0; tile < t1; ++tile) {
      const uint32_t p = static_cast<uint32_t>(tile) * kTile + tid;
      const bool valid = p < m;
#pragma unroll
      for (int j = 0; j < NB4; ++j) {
        T x = 0;
        if (j < n && valid) x = (X + static_cast<size_t>(j) * m)[p];
        const double xd = static_cast<double>(x);
        s1 += fabs(xd);
        s2 = fma(xd, xd, s2);
        nf += finite_val(x) ? 0.0 : 1.0;
        tileA[j * LDT + tid] = x;
      }
      gram_tile();
    }
  } else if constexpr (WARM) {
    // A_1 = X - S0 + Y0/mu; S0 and Y0 go to the buffers pass 1 reads
    const gptr<const T> S0 = as_global<T>(d.S0);
    const gptr<const T> Y0 = as_global<T>(d.Y0);
    const gptr<T> S1 = as_global<T>(d.S[0]);
    const gptr<T> Y1 = as_global<T>(d.Y[0]);
#pragma unroll 1
    for (int tile = t0; tile < t1; ++tile) {
      const uint32_t p = static_cast<uint32_t>(tile) * kTile + tid;
      const bool valid = p < m;
#pragma unroll
      for (int j = 0; j < NB4; ++j) {
        T a = 0;
        if (j < n && valid) {
          const size_t col = static_cast<size_t>(j) * m;
          const T x = (X + col)[p];
          const T s = d.S0 ? (S0 + col)[p] : T(0);
          const T y = d.Y0 ? (Y0 + col)[p] : T(0);
          (S1 + col)[p] = s;
          (Y1 + col)[p] = y;
          a = fma(y, imu, x - s);
        }
        tileA[j * LDT + tid] = a;
      }
      gram_tile();
    }
  } else {
#pragma unroll 1
    for (int tile = t0; tile < t1; ++tile) {
      const uint32_t p = static_cast<uint32_t>(tile) * kTile + tid;
      const int64_t mt = opaque(m);
      const bool valid = p < mt;
      T x[NB], y[NB], a[NB];
      {
        const gptr<const T> Xt = opaque(X), St = opaque(Sin), Yt = opaque(Yin);
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          x[j] = 0; y[j] = 0; a[j] = 0;
          if (j < n && valid) {
            const size_t col = static_cast<size_t>(j) * mt;
            T s = 0;
            x[j] = (Xt + col)[p];
            if (!first) {
              s = (St + col)[p];
              y[j] = (Yt + col)[p];
            }
            a[j] = fma(y[j], imu, x[j] - s);
          }
        }
      }
      // The projector's address is made opaque to the compiler per tile, so
      // its scalar loads stay inside the loop next to their uses instead of
      // being hoisted (NB^2 values would not fit the scalar registers).
      const cptr<T> P = as_const<T>(static_cast<const void*>(opaque(static_cast<const T*>(d.P))));
      const gptr<T> So_t = opaque(Sout), Yo_t = opaque(Yout);
#pragma unroll
      for (int j = 0; j < NB4; ++j) {
        T apj = 0;
        if (j < NB && j < n) {
          // Eq. 4 rebuild: l = sum_i a_i P_ij (P is zero outside n x n and
          // exactly symmetric; row j of P is contiguous for scalar loads).
          T l = 0;
#pragma unroll
          for (int i = 0; i < NB; ++i) l = fma(a[i], P[j * NB + i], l);
          const T tt = fma(y[j], imu, x[j]) - l;          // X - L + Y/mu
          const T sn_ = tt - clamp_sym(tt, gam);           // Eq. 5 shrink
          const T z = (x[j] - l) - sn_;                    // X - L - S
          const T yn_ = fma(mu, z, y[j]);                  // Eq. 6
          const double zd = static_cast<double>(z);
          r2 = fma(zd, zd, r2);
          apj = fma(yn_, imu, x[j] - sn_);                 // next X - S + Y/mu
          if (valid) {
            const size_t col = static_cast<size_t>(j) * mt;
            (So_t + col)[p] = sn_;
            (Yo_t + col)[p] = yn_;
          } else {
            apj = 0;
          }
        }
        tileA[j * LDT + tid] = apj;
      }
      gram_tile();
    }
  }

#ifdef RPCA_TRACE
  const int64_t t_tiles = RPCA_NOW();
#endif
  // Workgroup partial.  Scalars: wave shuffles, then the waves in order.
  // Gram blocks: lane-group sums in registers, then through LDS, where one
  // thread per block entry adds the Q group sums in chunk order.
  double sc[kScalars] = {r2, s1, s2, nf};
#pragma unroll
  for (int s = 0; s < kScalars; ++s) sc[s] = wave_sum(sc[s]);
  if ((tid & 63) == 0) {
#pragma unroll
    for (int s = 0; s < kScalars; ++s) wred[tid >> 6][s] = sc[s];
  }
  if (G >= 2) {
#pragma unroll
    for (int e = 0; e < 16; ++e) gacc[e] += quad_swap<kQuadXor1>(gacc[e]);
    if (G == 4) {
#pragma unroll
      for (int e = 0; e < 16; ++e) gacc[e] += quad_swap<kQuadXor2>(gacc[e]);
    }
  }
  if (gact && (gc & (G - 1)) == 0) {
    double* dst = red + (gblk * Q + gc / G) * kRedLd;
#pragma unroll
    for (int e = 0; e < 16; ++e) dst[e] = gacc[e];
  }
  __syncthreads();
  const gptr<double> part = as_global<double>(static_cast<void*>(
      d.partials + static_cast<size_t>(wi.slot) * d.pstride));
  for (int idx = tid; idx < nblk * 16; idx += kThreads) {
    const double* src = red + (idx >> 4) * Q * kRedLd + (idx & 15);
    double s = 0.0;
#pragma unroll 4
    for (int c = 0; c < Q; ++c) s += src[c * kRedLd];
    part[kScalars + idx] = s;
  }
  if (tid < kScalars) {
    double s = wred[0][tid];
#pragma unroll
    for (int w = 1; w < kThreads / 64; ++w) s += wred[w][tid];
    part[tid] = s;
  }
#ifdef RPCA_TRACE
  if (tid == 0 && d.wgtrace) {
    d.wgtrace[wi.slot * 4 + 0] = t_begin;
    d.wgtrace[wi.slot * 4 + 1] = t_tiles;
    d.wgtrace[wi.slot * 4 + 2] = RPCA_NOW();
  }
#else
  (void)t_begin;
#endif
}

template <typename T, int NB, bool MT>
__global__ void __launch_bounds__(kThreads)
k_finalize(const SolveDesc* __restrict__ descs, const WorkItem* __restrict__ items) {
  const int tid = threadIdx.x;
  const WorkItem wi = items[blockIdx.x];
  const SolveDesc& d = descs[wi.solve];
  const SolveState* st = d.st;
  if (st->status < 0) return;
  const int k = st->iter;
  const int n = d.n;
  const int64_t m = d.m;
  const gptr<const T> X = as_global<T>(d.X);
  const gptr<const T> Sprev = as_global<T>(static_cast<const void*>(d.S[(k + 1) & 1]));
  const gptr<const T> Yprev = as_global<T>(static_cast<const void*>(d.Y[(k + 1) & 1]));
  const gptr<const T> Sk = as_global<T>(static_cast<const void*>(d.S[k & 1]));
  const gptr<T> L = as_global<T>(d.Lout);
  const gptr<T> So = as_global<T>(d.Sout);
  const gptr<T> Yo = as_global<T>(d.Yout);
  const gptr<const T> Yk = as_global<T>(static_cast<const void*>(d.Y[k & 1]));
  const bool first = (k == 1) && !d.warm;
  const T imu = static_cast<T>(st->imu);
  const int t0 = wi.slot * d.tps;
  const int t1 = MT ? min(t0 + d.tps, d.tiles) : t0 + 1;
#pragma unroll 1
  for (int tile = t0; tile < t1; ++tile) {
    const uint32_t p = static_cast<uint32_t>(tile) * kTile + tid;
    if (p >= m) break;
    if (k == 0) {  // sum|X| == 0: L = S = 0 (and Y = 0)
      for (int j = 0; j < n; ++j) {
        const size_t col = static_cast<size_t>(j) * m;
        (L + col)[p] = T(0);
        (So + col)[p] = T(0);
        if (d.Yout) (Yo + col)[p] = T(0);
      }
      continue;
    }
    T a[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      a[j] = 0;
      if (j < n) {
        const size_t col = static_cast<size_t>(j) * m;
        const T x = (X + col)[p];
        T s = 0, y = 0;
        if (!first) {
          s = (Sprev + col)[p];
          y = (Yprev + col)[p];
        }
        a[j] = fma(y, imu, x - s);
      }
    }
    const cptr<T> P = as_const<T>(static_cast<const void*>(opaque(static_cast<const T*>(d.P))));
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (j < n) {
        T l = 0;
#pragma unroll
        for (int i = 0; i < NB; ++i) l = fma(a[i], P[j * NB + i], l);
        const size_t col = static_cast<size_t>(j) * m;
        (L + col)[p] = l;
        (So + col)[p] = (Sk + col)[p];
        if (d.Yout) (Yo + col)[p] = (Yk + col)[p];
      }
    }
  }
}

// Launch one register class (dispatch helper of the instantiation units).
template <typename T, int NB, bool MT>
hipError_t launch_stream_class(int mode, int grid, hipStream_t stream, const SolveDesc* descs,
                               const WorkItem* items) {
  const dim3 g(grid), b(kThreads);
  if (mode == kModeInit)
    RPCA_LAUNCH((k_stream<T, NB, kModeInit, MT>), g, b, 0, stream, descs, items);
  else if (mode == kModeUpdate)
    RPCA_LAUNCH((k_stream<T, NB, kModeUpdate, MT>), g, b, 0, stream, descs, items);
  else if (mode == kModeWarm)
    RPCA_LAUNCH((k_stream<T, NB, kModeWarm, MT>), g, b, 0, stream, descs, items);
  else
    RPCA_LAUNCH((k_finalize<T, NB, MT>), g, b, 0, stream, descs, items);
  return hipGetLastError();
}

}  // namespace rpca
