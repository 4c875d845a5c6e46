// MFMA streaming kernel of the RPCA iteration (paper Sec. II-A, Eqs. 4-6):
// FP32 storage for every frame class up to 144 frames and for every class in
// the split-BF16 precision variants; FP64 storage for the classes of 33 to
// 128 frames.
//
// A workgroup (8 wavefronts) walks a contiguous run of 64-row tiles of one
// solve.  Per tile:
//   1. load X, S, Y coalesced (lane = pixel row, wave w takes frames w,
//      w + waves, ...), keep X and Y in registers and put A = X - S + Y/mu
//      into an LDS tile stored frame-major; the next tile's loads are issued
//      right after, so they are in flight during the contractions;
//   2. rebuild L^T = P A^T on the matrix cores into a second LDS tile (P is
//      symmetric; FP64 storage keeps the products in registers until every
//      wave has read the A tile, then writes L over it, so one tile of
//      doubles fits the LDS); each 16-frame output block is shared by NW / NT16 waves
//      (by 16-row blocks), which keep their rows of P in registers for the
//      whole launch.  With more blocks than waves (144 frames) wave w owns
//      block w and the extra blocks are split by 16-row block over the first
//      waves;
//   3. read back each thread's L entries and apply the fused elementwise
//      step (shrink, dual update, residual, next A) exactly as the register
//      kernel does; the next A overwrites the A tile;
//   4. accumulate the Gram A'^T A' of the tile on the matrix cores; wave w
//      owns every NW-th 16 x 16 output block (upper triangle) and keeps it in
//      registers across the tiles of the workgroup.
// The workgroup writes one partial (scalars and Gram, in the 4 x 4 block
// layout of the other streaming kernels) at the end, so the reduction and
// eigensolve kernels are shared.
//
// Precision (PREC):
//   0  FP32 storage: rebuild with FP32 products and FP32 accumulation
//      (v_mfma_f32_16x16x4f32); Gram with exact FP64 products of the FP32
//      values and FP64 accumulation (v_mfma_f64_16x16x4f64), as in the
//      register kernel.  FP64 storage: both contractions on
//      v_mfma_f64_16x16x4f64;
//   1  both contractions as three BF16 products, hi*hi + hi*lo + lo*hi of the
//      split x = hi + lo (hi = bf16(x), lo = bf16(x - hi)), on
//      v_mfma_f32_16x16x32_bf16 with FP32 accumulation; the Gram is
//      accumulated in FP32 over each 64-row tile and in FP64 across tiles;
//   2  the same with the three-way split x = hi + mid + lo and the six
//      products whose order is at most 2^-16 relative to hi*hi (hi*hi,
//      hi*mid, mid*hi, hi*lo, mid*mid, lo*hi): about FP32 accuracy.
#pragma once

#include <type_traits>

#include "common.h"
#include "launch.h"

namespace rpca {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int R = kWideRows;  // rows per tile
// Frame-major LDS tiles with a row stride of 81 = 17 (mod 32): both MFMA
// operand patterns (16 frames x 4 rows and 4 frames x 16 rows per wave) then
// fall in distinct banks within each half-wave.
constexpr int LDA = R + 17;
// Wavefronts per workgroup.  (16 waves above 64 frames were measured slower:
// the 128-register cap of 1024-thread workgroups makes them spill.)
__host__ __device__ constexpr int waves_for(int) { return 8; }

__device__ inline float clamp_t(float v, float g) { return fminf(fmaxf(v, -g), g); }
__device__ inline double clamp_t(double v, double g) { return fmin(fmax(v, -g), g); }

__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = static_cast<__bf16>(x);
  lo = static_cast<__bf16>(x - static_cast<float>(hi));
}

__device__ inline void split3_bf16(float x, __bf16& hi, __bf16& mid, __bf16& lo) {
  hi = static_cast<__bf16>(x);
  const float r = x - static_cast<float>(hi);
  mid = static_cast<__bf16>(r);
  lo = static_cast<__bf16>(r - static_cast<float>(mid));
}

// Accumulate the split product sum of one 16x16x32 block: three products of
// the two-way split (X6 = false) or six of the three-way split, smallest
// terms first.
template <bool X6>
__device__ inline f4 mfma_split(const bf8& ah, const bf8& am, const bf8& al, const bf8& bh,
                                const bf8& bm, const bf8& bl, f4 acc) {
  if constexpr (X6) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm, acc, 0, 0, 0);
  } else {
    (void)am;
    (void)bm;
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
  }
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
}

template <bool X6>
__device__ inline void split_any(float x, __bf16& hi, __bf16& mid, __bf16& lo) {
  if constexpr (X6) {
    split3_bf16(x, hi, mid, lo);
  } else {
    split_bf16(x, hi, lo);
    mid = static_cast<__bf16>(0.0f);
  }
}

template <typename T, int NB, int PHASE, int PREC>
__global__ void __launch_bounds__(waves_for(NB) * 64)
k_wide(const SolveDesc* __restrict__ descs, const WorkItem* __restrict__ items) {
  static_assert(NB % 16 == 0 && NB <= 144, "frame class");
  constexpr bool F64 = std::is_same<T, double>::value;
  static_assert(!F64 || (PREC == 0 && NB <= 128), "FP64 storage: plain contractions, <= 128 frames");
  constexpr int NW = waves_for(NB);
  constexpr int NTH = NW * 64;
  constexpr int NQ = NB / NW;                           // frames per thread
  constexpr int NK4 = NB / 4;                           // f32 k-steps of the rebuild
  constexpr int NT16 = NB / 16;                         // 16-frame blocks
  constexpr bool X6 = PREC == 2;
  constexpr int NBK = PREC ? (NB + 31) / 32 * 32 : NB;  // contraction length of the rebuild
  constexpr int NKB = NBK / 32;                         // bf16 k-steps of the rebuild
  constexpr int NGT = NT16 * (NT16 + 1) / 2;            // Gram output blocks (upper)
  constexpr int MG = (NGT + NW - 1) / NW;               // ... per wave
  constexpr bool INIT = PHASE == kModeInit;
  constexpr bool WARM = PHASE == kModeWarm;
  constexpr bool FIN = PHASE == kModeFinalize;
  constexpr bool REB = !INIT && !WARM;  // passes that rebuild L
  // FP64: L overwrites the A tile after the rebuild (LS = At)
  __shared__ T At[NBK * LDA];
  __shared__ float Lt[REB && !F64 ? NB * LDA : 1];
  __shared__ double wred[NW][kScalars];
  // FP64 96-frame class: the projector rows in LDS instead of registers
  // (48 registers per lane that the update pass would otherwise spill;
  // 73.7 KB beside the 62.2 KB A tile).  Larger FP64 classes do not fit.
  constexpr bool PL = F64 && NB == 96 && REB;
  constexpr int LDP = NB + 1;
  __shared__ T Ps[PL ? NB * LDP : 1];

  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63;
  const WorkItem wi = items[blockIdx.x];
  const SolveDesc& d = descs[wi.solve];
  SolveState* st = d.st;
  int k = 0;
  if constexpr (WARM) {
    if (st->done || st->warm_stage != 1) return;
  }
  if constexpr (PHASE == kModeUpdate) {
    if (st->done) return;
    k = st->iter;
  }
  if constexpr (FIN) {
    if (st->status < 0) return;
    k = st->iter;
  }
  const int n = d.n;
  const int64_t m = d.m;
  const gptr<const T> X = as_global<T>(d.X);
  // update: read S_{k-1}, Y_{k-1}, write S_k, Y_k; finalize: read S_{k-1}, Y_{k-1}
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

  // zero the padding frames of the A tile once (never written afterwards)
  for (int idx = NB * LDA + tid; idx < NBK * LDA; idx += NTH) At[idx] = T(0);

  // Rebuild work: frame block t = w mod NT16 and every NREP-th 16-row block
  // of the tile starting at w / NT16, so all waves share the rebuild when the
  // class has fewer frame blocks than waves.  With more blocks than waves
  // (XTRA), wave w owns block w for every row block, and the 16-row blocks of
  // the extra blocks NW, NW+1, ... go one each to waves 0, 1, ...
  constexpr bool XTRA = NT16 > NW;
  static_assert(!XTRA || 4 * (NT16 - NW) <= NW, "extra frame blocks exceed the waves");
  constexpr int NOWN = XTRA ? 2 : 1;
  constexpr int NREP = XTRA ? 1 : NW / NT16;
  const int own_t[2] = {XTRA ? w : w % NT16, NW + (w >> 2)};
  const bool owns[2] = {XTRA || w < NT16 * NREP, XTRA && w < 4 * (NT16 - NW)};
  T pa[PREC || PL ? 1 : NOWN][PREC || PL ? 1 : NK4];
  bf8 ph[PREC ? NOWN : 1][PREC ? NKB : 1], pl[PREC ? NOWN : 1][PREC ? NKB : 1];
  bf8 pm[X6 ? NOWN : 1][X6 ? NKB : 1];
  if constexpr (REB) {
    const gptr<const T> P = as_global<T>(static_cast<const void*>(d.P));
#pragma unroll
    for (int o = 0; o < NOWN; ++o) {
      const int t = own_t[o];
      const int prow = 16 * (owns[o] ? t : 0) + (l & 15);
      if constexpr (PREC == 0) {
        if constexpr (!PL) {
#pragma unroll
          for (int kk = 0; kk < NK4; ++kk) pa[o][kk] = P[prow * NB + 4 * kk + (l >> 4)];
        }
      } else {
#pragma unroll
        for (int kk = 0; kk < NKB; ++kk) {
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int col = 32 * kk + 8 * (l >> 4) + e;
            const float v = col < NB ? static_cast<float>(P[prow * NB + col]) : 0.f;
            __bf16 h, md, lo;
            split_any<X6>(v, h, md, lo);
            ph[o][kk][e] = h;
            pl[o][kk][e] = lo;
            if constexpr (X6) pm[o][kk][e] = md;
          }
        }
      }
    }
  }

  if constexpr (PL) {  // read by the rebuild after the first tile's barrier
    const gptr<const T> P = as_global<T>(static_cast<const void*>(d.P));
    for (int idx = tid; idx < NB * NB; idx += NTH) Ps[(idx / NB) * LDP + idx % NB] = P[idx];
  }
  // Gram blocks owned by this wave and their accumulators.
  int gbi[MG], gbj[MG];
  d4 gacc[MG];
#pragma unroll
  for (int g = 0; g < MG; ++g) {
    const int idx = w + NW * g;
    int bj = 0;
    if (idx < NGT) {
      while ((bj + 1) * (bj + 2) / 2 <= idx) ++bj;
    }
    gbj[g] = bj;
    gbi[g] = idx < NGT ? idx - bj * (bj + 1) / 2 : 0;
    gacc[g] = d4{0.0, 0.0, 0.0, 0.0};
  }
  double r2 = 0.0, s1 = 0.0, s2 = 0.0, nf = 0.0;

  const int t0 = wi.slot * d.tps;
  const int t1 = min(t0 + d.tps, d.tiles);
  if constexpr (FIN) {
    if (k == 0) {  // sum|X| == 0: L = S = 0 (no projector was computed)
      for (int tile = t0; tile < t1; ++tile) {
        const int64_t p = static_cast<int64_t>(tile) * R + l;
        if (p >= m) continue;
        for (int q = 0; q < NQ; ++q) {
          const int j = w + NW * q;
          if (j >= n) continue;
          const size_t off = static_cast<size_t>(j) * static_cast<size_t>(m) + static_cast<size_t>(p);
          as_global<T>(d.Lout)[off] = T(0);
          as_global<T>(d.Sout)[off] = T(0);
          if (d.Yout) as_global<T>(d.Yout)[off] = T(0);
        }
      }
      return;
    }
  }
  // Raw loads of one tile: X, and S_{k-1}, Y_{k-1} after the first iteration
  // (the given S0, Y0 in the warm pass).
  const bool read_sy = REB && k >= 1 && !first;
  const gptr<const T> S0 = as_global<T>(d.S0);
  const gptr<const T> Y0 = as_global<T>(d.Y0);
  auto load_tile = [&](int tile, T* xr, T* sr, T* yr) {
    const int64_t p = static_cast<int64_t>(tile) * R + l;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int j = w + NW * q;
      xr[q] = T(0);
      sr[q] = T(0);
      yr[q] = T(0);
      if (j < n && p < m) {
        const size_t off = static_cast<size_t>(j) * static_cast<size_t>(m) + static_cast<size_t>(p);
        xr[q] = X[off];
        if constexpr (WARM) {
          if (d.S0) sr[q] = S0[off];
          if (d.Y0) yr[q] = Y0[off];
        } else if (read_sy) {
          sr[q] = Sin[off];
          yr[q] = Yin[off];
        }
      }
    }
  };
  // With few frames per thread the next tile's loads are issued before the
  // current tile's contractions, so they are in flight meanwhile (up to 40
  // bytes of each of X, S, Y per thread).
  constexpr bool PF = NQ * static_cast<int>(sizeof(T)) <= 40;
  T xn[PF ? NQ : 1], sn_[PF ? NQ : 1], yn[PF ? NQ : 1];
  if constexpr (PF) {
    if (t0 < t1) load_tile(t0, xn, sn_, yn);
  }
  for (int tile = t0; tile < t1; ++tile) {
    const int64_t p = static_cast<int64_t>(tile) * R + l;
    const bool valid = p < m;
    T x[NQ], y[NQ], sv[NQ];
    // 1. load, A tile
    if constexpr (PF) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        x[q] = xn[q];
        sv[q] = sn_[q];
        y[q] = yn[q];
      }
    } else {
      load_tile(tile, x, sv, y);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int j = w + NW * q;
      T a = T(0);
      if (j < n && valid) {
        if constexpr (INIT) {
          const double xd = static_cast<double>(x[q]);
          s1 += fabs(xd);
          s2 = fma(xd, xd, s2);
          nf += __builtin_isfinite(x[q]) ? 0.0 : 1.0;
          a = x[q];
        } else {
          a = fma(y[q], imu, x[q] - sv[q]);
          if constexpr (WARM) {  // the buffers the first update pass reads
            const size_t off = static_cast<size_t>(j) * static_cast<size_t>(m) + static_cast<size_t>(p);
            as_global<T>(d.S[0])[off] = sv[q];
            as_global<T>(d.Y[0])[off] = y[q];
          }
        }
      }
      At[j * LDA + l] = a;
    }
    if constexpr (PF) {
      if (tile + 1 < t1) load_tile(tile + 1, xn, sn_, yn);
    }
    __syncthreads();

    if constexpr (REB) {
      // 2. rebuild L^T = P A^T into Lt.  FP64 writes L over the A tile: the
      // waves take their 16-row blocks in steps (all waves step c together),
      // and a barrier after the products of a step lets them write that
      // step's rows, which no later step reads.
      if constexpr (F64) {
        constexpr int MRB = (R / 16 + NREP - 1) / NREP;  // steps
        const int t = own_t[0];
        const int rb0 = w / NT16;
#pragma unroll
        for (int c = 0; c < MRB; ++c) {
          const int rb = rb0 + c * NREP;
          const bool act = owns[0] && rb < R / 16;
          d4 acc = {0.0, 0.0, 0.0, 0.0};
          if (act) {
#pragma unroll
            for (int kk = 0; kk < NK4; ++kk) {
              const double b = At[(4 * kk + (l >> 4)) * LDA + 16 * rb + (l & 15)];
              double a;
              if constexpr (PL) a = Ps[(16 * t + (l & 15)) * LDP + 4 * kk + (l >> 4)];
              else a = pa[0][kk];
              acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
          }
          __syncthreads();  // every wave is past its reads of this step's rows
          if (act) {
            // f64 MFMA: lane l, register r holds entry (l/16 + 4r, l%16)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              At[(16 * t + (l >> 4) + 4 * r) * LDA + 16 * rb + (l & 15)] = acc[r];
          }
        }
      } else {
#pragma unroll
        for (int o = 0; o < NOWN; ++o) {
          const int t = own_t[o];
          if (owns[o]) {
            const int rb0 = o == 0 ? (XTRA ? 0 : w / NT16) : (w & 3);
            const int rstep = o == 0 ? NREP : R / 16;
#pragma unroll 1
            for (int rb = rb0; rb < R / 16; rb += rstep) {
              f4 acc = {0.f, 0.f, 0.f, 0.f};
              if constexpr (PREC == 0) {
#pragma unroll
                for (int kk = 0; kk < NK4; ++kk) {
                  const float b = At[(4 * kk + (l >> 4)) * LDA + 16 * rb + (l & 15)];
                  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(pa[o][kk], b, acc, 0, 0, 0);
                }
              } else {
#pragma unroll
                for (int kk = 0; kk < NKB; ++kk) {
                  bf8 bh, bm, bl;
#pragma unroll
                  for (int e = 0; e < 8; ++e) {
                    const float v = At[(32 * kk + 8 * (l >> 4) + e) * LDA + 16 * rb + (l & 15)];
                    __bf16 h, md, lo;
                    split_any<X6>(v, h, md, lo);
                    bh[e] = h;
                    bm[e] = md;
                    bl[e] = lo;
                  }
                  acc = mfma_split<X6>(ph[o][kk], X6 ? pm[o][kk] : bm, pl[o][kk], bh, bm, bl, acc);
                }
              }
#pragma unroll
              for (int r = 0; r < 4; ++r)
                Lt[(16 * t + 4 * (l >> 4) + r) * LDA + 16 * rb + (l & 15)] = acc[r];
            }
          }
        }
      }
      __syncthreads();

      // 3. elementwise step (or the final L); FP64 reads L and writes the
      // next A at the same place of the A tile (the thread's own entries)
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int j = w + NW * q;
        T lv;
        if constexpr (F64) lv = At[j * LDA + l];
        else lv = Lt[j * LDA + l];
        T apj = T(0);
        if (j < n && valid) {
          const size_t off = static_cast<size_t>(j) * static_cast<size_t>(m) + static_cast<size_t>(p);
          if constexpr (FIN) {
            as_global<T>(d.Lout)[off] = lv;
            as_global<T>(d.Sout)[off] = as_global<T>(static_cast<const void*>(d.S[k & 1]))[off];
            if (d.Yout)
              as_global<T>(d.Yout)[off] = as_global<T>(static_cast<const void*>(d.Y[k & 1]))[off];
          } else {
            const T tt = fma(y[q], imu, x[q]) - lv;                 // X - L + Y/mu
            const T sn = tt - clamp_t(tt, gam);                     // Eq. 5 shrink
            const T z = (x[q] - lv) - sn;                           // X - L - S
            const T yn = fma(mu, z, y[q]);                          // Eq. 6
            const double zd = static_cast<double>(z);
            r2 = fma(zd, zd, r2);
            apj = fma(yn, imu, x[q] - sn);                          // next X - S + Y/mu
            Sout[off] = sn;
            Yout[off] = yn;
          }
        }
        if constexpr (!FIN) At[j * LDA + l] = apj;
      }
      __syncthreads();
    }

    // 4. Gram of the tile
    if constexpr (!FIN) {
#pragma unroll
      for (int g = 0; g < MG; ++g) {
        if (w + NW * g < NGT) {
          const T* u = At + (16 * gbi[g] + (l & 15)) * LDA;
          const T* v = At + (16 * gbj[g] + (l & 15)) * LDA;
          if constexpr (PREC == 0) {
#pragma unroll
            for (int kk = 0; kk < R / 4; ++kk) {
              const double a = static_cast<double>(u[4 * kk + (l >> 4)]);
              const double b = static_cast<double>(v[4 * kk + (l >> 4)]);
              gacc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, gacc[g], 0, 0, 0);
            }
          } else {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < R / 32; ++kk) {
              bf8 ah, am, al, bh, bm, bl;
#pragma unroll
              for (int e = 0; e < 8; ++e) {
                __bf16 h, md, lo;
                split_any<X6>(u[32 * kk + 8 * (l >> 4) + e], h, md, lo);
                ah[e] = h;
                am[e] = md;
                al[e] = lo;
                split_any<X6>(v[32 * kk + 8 * (l >> 4) + e], h, md, lo);
                bh[e] = h;
                bm[e] = md;
                bl[e] = lo;
              }
              acc = mfma_split<X6>(ah, am, al, bh, bm, bl, acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) gacc[g][r] += static_cast<double>(acc[r]);
          }
        }
      }
      __syncthreads();
    }
  }

  if constexpr (!FIN) {
    // Partial of the workgroup: scalars by wave then in wave order; Gram
    // entries straight from the accumulators (each entry has one owner).
    double sc[kScalars] = {r2, s1, s2, nf};
#pragma unroll
    for (int s = 0; s < kScalars; ++s) sc[s] = wave_sum_d(sc[s]);
    if (l == 0) {
#pragma unroll
      for (int s = 0; s < kScalars; ++s) wred[w][s] = sc[s];
    }
    const gptr<double> part = as_global<double>(static_cast<void*>(d.partials + static_cast<size_t>(wi.slot) * d.pstride));
#pragma unroll
    for (int g = 0; g < MG; ++g) {
      if (w + NW * g < NGT) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          // f64 MFMA rows interleave (l/16 + 4r); f32 MFMA rows are blocked (4(l/16) + r)
          const int i = 16 * gbi[g] + (PREC == 0 ? (l >> 4) + 4 * r : 4 * (l >> 4) + r);
          const int j = 16 * gbj[g] + (l & 15);
          const int bi4 = i >> 2, bj4 = j >> 2;
          if (bi4 <= bj4)
            part[kScalars + (bj4 * (bj4 + 1) / 2 + bi4) * 16 + (i & 3) * 4 + (j & 3)] = gacc[g][r];
        }
      }
    }
    __syncthreads();
    if (tid < kScalars) {
      double sum = wred[0][tid];
#pragma unroll
      for (int v = 1; v < NW; ++v) sum += wred[v][tid];
      part[tid] = sum;
    }
  }
}

}  // namespace
}  // namespace rpca
