// FP64 eigensolve and singular value thresholding weights for windows of 65
// to 144 frames (paper Sec. II-A, Eq. 4; the paper's own reference windows
// have 132 frames).
//
// Same method as the LDS eigensolver of the smaller classes: cyclic
// two-sided Jacobi on the n x n Gram G = A^T A with the round-robin parallel
// ordering, rotations of the smaller angle, and P = V diag(w) V^T with
// w_i = max(sigma_i - tau, 0) / sigma_i.  At these sizes two copies of G and
// V do not fit in the 160 KB of LDS, so the rotations are applied in place:
//
//   * G is kept as its packed upper triangle.  In one round the disjoint
//     pairs (p_k, q_k) split G into 2 x 2 blocks, and block (k1, k2) of
//     J^T G J depends only on block (k1, k2) of G, so each thread owns whole
//     blocks and overwrites them;
//   * V is kept in full; row i of V J depends only on row i, so each thread
//     owns (row, pair) items and overwrites V[i][p], V[i][q].  Up to 112
//     frames V sits in LDS beside G; in the 144-frame class (packed G alone
//     takes 83.5 KB) it stays in the solve's V buffer in global memory.
//     FP64 solves, and FP32 solves of more than 136 frames, rotate it there
//     in place (the barriers of each round order the accesses, and the
//     166 KB stay in L2).  Warm-started FP32 solves of up to 136 frames
//     leave V fixed during the sweeps and accumulate the rotations as an
//     increment D in LDS, in FP32 (V J_1 J_2 ... = V (I + D)); each rotation
//     adds terms of the size of its angle to D, so D's rounding shrinks with
//     the angles as the iteration settles.  One product V <- V + V D on the
//     f64 matrix cores ends the eigensolve.  The cold start, whose rotations
//     build all of V, rotates V in place;
//   * a round is [apply the round's rotations] barrier [the first wave
//     computes the next round's rotations from the updated G] barrier.
//
// Warm start: from the second step on, the rotations start from the previous
// step's eigenvectors V, on G~ = V^T G V, which is nearly diagonal once the
// iteration settles.  The two products run on the f64 matrix cores
// (W = G V goes through a per-solve global scratch buffer, since LDS holds G
// and V already).  For FP64 solves, and for FP32 solves that accumulate an
// FP32 increment, V is first brought back to orthogonality by one
// Newton-Schulz step V <- V (3I - V^T V) / 2 (also on the matrix cores); for
// the other FP32 solves the rounding of the FP64 rotations stays far below
// the FP32 rounding of the data and the step is skipped.  With V in global
// memory the projector P = V diag(w) V^T is also formed on the f64 matrix
// cores.
#include <type_traits>

#include "common.h"
#include "eig_common.h"
#include "launch.h"

namespace rpca {
namespace {

using namespace eigk;

// FP32 solves of the device-memory class up to this many frames accumulate
// their rotations as an FP32 increment in LDS (74.5 KB beside packed G).
constexpr int kEigIncMaxN = 136;

__device__ inline int pk(int i, int j) {  // packed upper index, i <= j
  return j * (j + 1) / 2 + i;
}
__device__ inline int pks(int i, int j) { return i <= j ? pk(i, j) : pk(j, i); }

template <typename T, int NMAX, int NT>
__global__ void __launch_bounds__(NT)
k_eig_wide(const SolveDesc* __restrict__ descs, const int32_t* __restrict__ ids) {
  constexpr bool VG = NMAX > kEigWideMaxN;  // V in global memory
  // FP32 solves of up to kEigIncMaxN frames in the device-memory class keep
  // V fixed during the sweeps and accumulate the sweeps' rotations as an
  // increment D (V J_1 J_2 ... = V (I + D)) in LDS, in FP32
  constexpr bool VI = VG && std::is_same<T, float>::value;
  constexpr int LDD = kEigIncMaxN + 1;
  constexpr int NPK = NMAX * (NMAX + 1) / 2;
  constexpr int LDV = NMAX + 1;
  constexpr int NPM = NMAX / 2;                               // pairs per round at most
  constexpr int NBLK = NPM * (NPM + 1) / 2;                   // 2x2 blocks (k1 <= k2)
  constexpr int MB = (NBLK + NT - 1) / NT;                    // blocks per thread
  static_assert(NMAX % 2 == 0, "even class size");
  __shared__ double Gp[NPK];
  __shared__ double Vs[VG ? 1 : NMAX * LDV];
  __shared__ float Ds[VI ? kEigIncMaxN * LDD : 1];
  __shared__ int tpq[NPM];      // p | q << 8
  __shared__ double2 tcs[NPM];  // (c, s): one 16-byte read per pair
  __shared__ double tdt[NPM];
  __shared__ double w[NMAX];
  __shared__ double scal[kScalars];
  __shared__ int s_go;
  __shared__ double s_tau;

  const int tid = threadIdx.x;
  const SolveDesc& d = descs[ids[blockIdx.x]];
  SolveState* st = d.st;
  if (st->done) return;
#ifdef RPCA_TRACE
  int64_t tprev = RPCA_NOW();
#define EIG_MARK(i)                               \
  do {                                            \
    if (tid == 0) {                               \
      const int64_t tnow_ = RPCA_NOW();           \
      st->trace[i] += tnow_ - tprev;              \
      tprev = tnow_;                              \
    }                                             \
  } while (0)
#else
#define EIG_MARK(i) \
  do {              \
  } while (0)
#endif
  const int n = d.n;
  const int nb = d.nb;
  const int kd = st->iter;
  // read now (thread 0 runs the control step), in flight during the reduction
  double pf_nXF2 = 0.0, pf_tau = 0.0;
  if (tid == 0) {
    pf_nXF2 = st->nXF2;
    pf_tau = st->tau;
  }

  const bool warm = kd > 0;
  // (warm starts only: the cold start's rotations build all of V, and D
  // would be of order one)
  const bool vinc = VI && warm && n <= kEigIncMaxN;
  // V rows: LDS (stride LDV) or the solve's V buffer (stride nb, nb x nb,
  // zero outside n x n)
  const gptr<double> Vg = as_global<double>(static_cast<void*>(d.V));
  for (int idx = tid; idx < NPK; idx += NT) Gp[idx] = 0.0;
  if constexpr (VG) {
    if (!warm) {
      for (int idx = tid; idx < nb * nb; idx += NT) {
        const int i = idx / nb, j = idx - (idx / nb) * nb;
        Vg[idx] = (i == j && i < n) ? 1.0 : 0.0;
      }
    }
    if (vinc)
      for (int idx = tid; idx < kEigIncMaxN * LDD; idx += NT) Ds[idx] = 0.0f;
  } else {
    for (int idx = tid; idx < NMAX * LDV; idx += NT) {
      const int i = idx / LDV, j = idx - (idx / LDV) * LDV;
      double v = (i == j && i < n) ? 1.0 : 0.0;
      if (warm && i < n && j < n) v = d.V[i * nb + j];
      Vs[idx] = v;
    }
  }
  if (tid < NMAX) w[tid] = 0.0;
  __syncthreads();

  // 0. Sum the group partials of the streaming pass in group order; the Gram
  // goes into the packed upper triangle.
  {
    const int nblk = gram_blocks((n + 3) >> 2);
    const int nent = kScalars + nblk * 16;
    constexpr int kChunk = 16;
    for (int idx = tid; idx < nent; idx += NT) {
      double sum = 0.0;
      for (int q0 = 0; q0 < d.groups; q0 += kChunk) {
        const int c = min(kChunk, d.groups - q0);
        double v[kChunk];
#pragma unroll
        for (int q = 0; q < kChunk; ++q)
          v[q] = q < c ? d.gpartials[static_cast<size_t>(q0 + q) * d.pstride + idx] : 0.0;
#pragma unroll
        for (int q = 0; q < kChunk; ++q)
          if (q < c) sum += v[q];
      }
      if (idx < kScalars) {
        scal[idx] = sum;
      } else {
        const int g = idx - kScalars;
        const int blk = g >> 4, e = g & 15;
        int bj = 0;
        while ((bj + 1) * (bj + 2) / 2 <= blk) ++bj;
        const int bi = blk - bj * (bj + 1) / 2;
        const int i = 4 * bi + (e >> 2), j = 4 * bj + (e & 3);
        if (i <= j && j < n) Gp[pk(i, j)] = sum;
      }
    }
  }
  __syncthreads();

  if (tid == 0) {
    double t = 0.0;
    s_go = control_step(d, st, scal, kd, pf_nXF2, pf_tau, t);
    s_tau = t;
  }
  __syncthreads();
  if (!s_go) return;
  EIG_MARK(0);
  const double tau = s_tau;

  if (warm) {
    // W = G V (every 16 x 16 block) into the scratch buffer, then the upper
    // blocks of G~ = V^T W, written over G once every wave is past its reads
    // of G.  The f64 MFMA result of lane l, register r is entry
    // (l/16 + 4r, l%16) of the 16 x 16 block.
    typedef double d4 __attribute__((ext_vector_type(4)));
    constexpr int NWV = NT / 64;
    constexpr int NT16 = NMAX / 16;
    constexpr int NUT = NT16 * (NT16 + 1) / 2;
    constexpr int MT = (NUT + NWV - 1) / NWV;
    const int wv = tid >> 6, l = tid & 63;
    const gptr<double> Wg = as_global<double>(static_cast<void*>(d.escratch));
    // with V in global memory the products stop at nb (V is nb x nb)
    const int nt16 = VG ? nb / 16 : NT16;
    if (std::is_same<T, double>::value || vinc) {
      // FP64 solves, and FP32 solves that accumulate an FP32 increment: one
      // Newton-Schulz step V <- V (3I - V^T V) / 2 first, so the rounding of
      // the rotations does not accumulate over the solve.
      // C = V^T V goes to the scratch; each wave keeps its blocks of V C in
      // registers until every wave has read V, then writes its entries of
      // the new V (each entry has one owner).
      auto vat = [&](int i, int j) -> double {
        return VG ? static_cast<double>(Vg[i * nb + j]) : Vs[i * LDV + j];
      };
      for (int t = wv; t < nt16 * nt16; t += NWV) {
        const int bi = t / nt16, bj = t - (t / nt16) * nt16;
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int kk = 0; kk < nt16 * 4; ++kk) {
          const int kq = 4 * kk + (l >> 4);
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(vat(kq, 16 * bi + (l & 15)),
                                                     vat(kq, 16 * bj + (l & 15)), acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) Wg[(16 * bi + (l >> 4) + 4 * r) * NMAX + 16 * bj + (l & 15)] = acc[r];
      }
      __syncthreads();
      constexpr int MV = (NT16 * NT16 + NWV - 1) / NWV;
      d4 vc[MV];
#pragma unroll
      for (int q = 0; q < MV; ++q) {
        const int t = wv + q * NWV;
        vc[q] = d4{0.0, 0.0, 0.0, 0.0};
        if (t < nt16 * nt16) {
          const int bi = t / nt16, bj = t - (t / nt16) * nt16;
#pragma unroll 4
          for (int kk = 0; kk < nt16 * 4; ++kk) {
            const int kq = 4 * kk + (l >> 4);
            vc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(vat(16 * bi + (l & 15), kq),
                                                         Wg[kq * NMAX + 16 * bj + (l & 15)], vc[q], 0, 0, 0);
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < MV; ++q) {
        const int t = wv + q * NWV;
        if (t < nt16 * nt16) {
          const int bi = t / nt16, bj = t - (t / nt16) * nt16;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = 16 * bi + (l >> 4) + 4 * r, j = 16 * bj + (l & 15);
            const double v1 = fma(-0.5, vc[q][r], 1.5 * vat(i, j));
            if constexpr (VG) Vg[i * nb + j] = v1;
            else Vs[i * LDV + j] = v1;
          }
        }
      }
      __syncthreads();
    }
    for (int t = wv; t < nt16 * nt16; t += NWV) {
      const int bi = t / nt16, bj = t - (t / nt16) * nt16;
      d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
      for (int kk = 0; kk < nt16 * 4; ++kk) {
        const int kq = 4 * kk + (l >> 4);
        const double a = Gp[pks(16 * bi + (l & 15), kq)];
        const double b = VG ? Vg[kq * nb + 16 * bj + (l & 15)] : Vs[kq * LDV + 16 * bj + (l & 15)];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) Wg[(16 * bi + (l >> 4) + 4 * r) * NMAX + 16 * bj + (l & 15)] = acc[r];
    }
    __syncthreads();
    d4 gt[MT];
    int tbi[MT], tbj[MT];
#pragma unroll
    for (int q = 0; q < MT; ++q) {
      const int t = wv + q * NWV;
      int bj = 0;
      if (t < NUT) {
        while ((bj + 1) * (bj + 2) / 2 <= t) ++bj;
      }
      tbj[q] = bj;
      tbi[q] = t < NUT ? t - bj * (bj + 1) / 2 : 0;
      gt[q] = d4{0.0, 0.0, 0.0, 0.0};
      if (t < NUT && 16 * bj < nt16 * 16) {
#pragma unroll 4
        for (int kk = 0; kk < nt16 * 4; ++kk) {
          const int kq = 4 * kk + (l >> 4);
          const double a = VG ? Vg[kq * nb + 16 * tbi[q] + (l & 15)] : Vs[kq * LDV + 16 * tbi[q] + (l & 15)];
          const double b = Wg[kq * NMAX + 16 * bj + (l & 15)];
          gt[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, gt[q], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < MT; ++q) {
      if (wv + q * NWV < NUT && 16 * tbj[q] < nt16 * 16) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * tbi[q] + (l >> 4) + 4 * r, j = 16 * tbj[q] + (l & 15);
          if (i <= j) Gp[pk(i, j)] = gt[q][r];
        }
      }
    }
    __syncthreads();
  }

  EIG_MARK(1);
  const int N2 = n + (n & 1);
  const int M = N2 - 1;
  const int NP = N2 / 2;
  const int nblk2 = NP * (NP + 1) / 2;

  // Owned 2x2 blocks (pair indices k1 <= k2) and V items (row, pair).
  // 2x2 blocks packed as k1 | k2 << 8
  int bk[MB];
#pragma unroll
  for (int q = 0; q < MB; ++q) {
    const int b = tid + q * NT;
    int k2 = 0;
    if (b < nblk2) {
      while ((k2 + 1) * (k2 + 2) / 2 <= b) ++k2;
    }
    bk[q] = (b < nblk2 ? b - k2 * (k2 + 1) / 2 : 0) | (k2 << 8);
  }
  // V items: a thread rotates one pair vk (its rotation read once per round)
  // in rows vr0, vr0 + vrs, ... (vrs = NT / NP threads share a pair).  In LDS
  // the threads of a pair are consecutive and take consecutive rows, so the
  // lanes of a wave hit distinct banks; in device memory consecutive threads
  // take consecutive pairs of one row, which touches fewer cache lines.
  const int vrs = NP > 0 ? NT / NP : 1;
  const bool vlds = !VG || vinc;
  const int vk = NP > 0 ? (vlds ? tid / vrs : tid % NP) : 0;
  const int vr0 = NP > 0 ? (vlds ? tid - (tid / vrs) * vrs : tid / NP) : n;
  const bool vact = NP > 0 && (vlds ? vk < NP : vr0 < vrs);

  // Rotations of round r for pairs handled by the first wave.
  auto make_round = [&](int r) {
    if (tid < NP) {
      int p, q;
      pair_indices(r, tid, N2, p, q);
      double c = 1.0, s = 0.0, dt = 0.0;
      if (q < n) make_rotation<T>(Gp[pk(p, p)], Gp[pk(q, q)], Gp[pk(p, q)], c, s, dt);
      tpq[tid] = p | (q << 8);
      tcs[tid] = make_double2(c, s);
      tdt[tid] = dt;
    }
  };

  int sweeps = 0;
  for (; sweeps < kMaxSweeps && n > 1; ++sweeps) {
    int need = 0;
    for (int idx = tid; idx < n * (n + 1) / 2; idx += NT) {
      int j = 0;
      while ((j + 1) * (j + 2) / 2 <= idx) ++j;
      const int i = idx - j * (j + 1) / 2;
      if (i < j && off_diag_large<T>(Gp[idx], Gp[pk(i, i)], Gp[pk(j, j)])) need = 1;
    }
    make_round(0);
    if (!__syncthreads_or(need)) break;
    for (int r = 0; r < M; ++r) {
      // apply round r: G blocks and V items, in place.  The items of a
      // thread are disjoint from each other (and from every other thread's),
      // so all reads of a group of items are issued before its writes;
      // otherwise each read would wait behind the previous item's write.
      double gv[MB][4];
      int gi[MB][4], gmode[MB];
#pragma unroll
      for (int q = 0; q < MB; ++q) {
        gmode[q] = 0;
        if (tid + q * NT < nblk2) {
          const int k1 = bk[q] & 0xff, k2 = bk[q] >> 8;
          const int pq1 = tpq[k1], pq2 = tpq[k2];
          const int p1 = pq1 & 0xff, q1 = pq1 >> 8, p2 = pq2 & 0xff, q2 = pq2 >> 8;
          const double s1 = tcs[k1].y, s2 = tcs[k2].y;
          if (k1 == k2) {
            if (s1 != 0.0) {
              gmode[q] = 1;
              gi[q][0] = pk(p1, p1);
              gi[q][1] = pk(q1, q1);
              gi[q][2] = pk(p1, q1);
              gv[q][0] = Gp[gi[q][0]];
              gv[q][1] = Gp[gi[q][1]];
            }
          } else if (s1 != 0.0 || s2 != 0.0) {
            gmode[q] = 2;
            gi[q][0] = pks(p1, p2);
            gi[q][1] = pks(p1, q2);
            gi[q][2] = pks(q1, p2);
            gi[q][3] = pks(q1, q2);
#pragma unroll
            for (int e = 0; e < 4; ++e) gv[q][e] = Gp[gi[q][e]];
          }
        }
      }
#pragma unroll
      for (int q = 0; q < MB; ++q) {
        if (gmode[q] == 1) {
          const double dt = tdt[bk[q] & 0xff];
          Gp[gi[q][0]] = gv[q][0] - dt;
          Gp[gi[q][1]] = gv[q][1] + dt;
          Gp[gi[q][2]] = 0.0;
        } else if (gmode[q] == 2) {
          const int k1 = bk[q] & 0xff, k2 = bk[q] >> 8;
          const double2 cs1 = tcs[k1], cs2 = tcs[k2];
          const double c1 = cs1.x, s1 = cs1.y, c2 = cs2.x, s2 = cs2.y;
          const double b_pp = gv[q][0], b_pq = gv[q][1], b_qp = gv[q][2], b_qq = gv[q][3];
          // T = B J2 (columns p2, q2), then J1^T T (rows p1, q1)
          const double t_pp = fma(c2, b_pp, -s2 * b_pq), t_pq = fma(s2, b_pp, c2 * b_pq);
          const double t_qp = fma(c2, b_qp, -s2 * b_qq), t_qq = fma(s2, b_qp, c2 * b_qq);
          Gp[gi[q][0]] = fma(c1, t_pp, -s1 * t_qp);
          Gp[gi[q][1]] = fma(c1, t_pq, -s1 * t_qq);
          Gp[gi[q][2]] = fma(s1, t_pp, c1 * t_qp);
          Gp[gi[q][3]] = fma(s1, t_pq, c1 * t_qq);
        }
      }
      constexpr int VC = 4;  // V rows read together
      if (vinc) {
        // D <- D J + (J - I) for the pair's plane rotation J, with J - I
        // written through c - 1 and s, so every term added to D is of the
        // size of the rotation angle and the FP32 rounding scales with it
        const double2 csk = vact ? tcs[vk] : make_double2(1.0, 0.0);
        if (csk.y != 0.0) {
          const float sk = static_cast<float>(csk.y);
          const float cm = static_cast<float>(csk.x - 1.0);
          const int pqk = tpq[vk];
          const int p = pqk & 0xff, qq = pqk >> 8;
          for (int i0 = vr0; i0 < n; i0 += VC * vrs) {
            float dp[VC], dq[VC];
#pragma unroll
            for (int u = 0; u < VC; ++u) {
              const int i = i0 + u * vrs;
              dp[u] = 0.0f;
              dq[u] = 0.0f;
              if (i < n) {
                dp[u] = Ds[i * LDD + p];
                dq[u] = Ds[i * LDD + qq];
              }
            }
#pragma unroll
            for (int u = 0; u < VC; ++u) {
              const int i = i0 + u * vrs;
              if (i < n) {
                const float ep = (i == p ? cm : 0.0f) - (i == qq ? sk : 0.0f);
                const float eq = (i == p ? sk : 0.0f) + (i == qq ? cm : 0.0f);
                Ds[i * LDD + p] = dp[u] + (fmaf(cm, dp[u], -sk * dq[u]) + ep);
                Ds[i * LDD + qq] = dq[u] + (fmaf(sk, dp[u], cm * dq[u]) + eq);
              }
            }
          }
        }
      } else if (vact && tcs[vk].y != 0.0) {
        const double2 csk = tcs[vk];
        const double sk = csk.y, ck = csk.x;
        const int pqk = tpq[vk];
        const int p = pqk & 0xff, qq = pqk >> 8;
        for (int i0 = vr0; i0 < n; i0 += VC * vrs) {
          double vp[VC], vq[VC];
#pragma unroll
          for (int u = 0; u < VC; ++u) {
            const int i = i0 + u * vrs;
            vp[u] = 0.0;
            vq[u] = 0.0;
            if (i < n) {
              if constexpr (VG) {
                const gptr<double> row = Vg + static_cast<size_t>(i) * nb;
                vp[u] = row[p];
                vq[u] = row[qq];
              } else {
                vp[u] = Vs[i * LDV + p];
                vq[u] = Vs[i * LDV + qq];
              }
            }
          }
#pragma unroll
          for (int u = 0; u < VC; ++u) {
            const int i = i0 + u * vrs;
            if (i < n) {
              const double np_ = fma(ck, vp[u], -sk * vq[u]);
              const double nq_ = fma(sk, vp[u], ck * vq[u]);
              if constexpr (VG) {
                const gptr<double> row = Vg + static_cast<size_t>(i) * nb;
                row[p] = np_;
                row[qq] = nq_;
              } else {
                Vs[i * LDV + p] = np_;
                Vs[i * LDV + qq] = nq_;
              }
            }
          }
        }
      }
      __syncthreads();
      if (r + 1 < M) make_round(r + 1);
      __syncthreads();
    }
  }

  EIG_MARK(2);
  if (vinc && sweeps > 0) {
    // V <- V + V D on the f64 matrix cores; each wave keeps its 16 x 16
    // blocks in registers until every wave has read V, then adds them to its
    // entries of V (each entry has one owner)
    typedef double d4 __attribute__((ext_vector_type(4)));
    constexpr int NWV = NT / 64;
    constexpr int NT16 = NMAX / 16;
    constexpr int MV = (NT16 * NT16 + NWV - 1) / NWV;
    const int wv = tid >> 6, l = tid & 63;
    const int nt16 = nb / 16;
    d4 vd[MV];
#pragma unroll
    for (int q = 0; q < MV; ++q) {
      const int t = wv + q * NWV;
      vd[q] = d4{0.0, 0.0, 0.0, 0.0};
      if (t < nt16 * nt16) {
        const int bi = t / nt16, bj = t - (t / nt16) * nt16;
        const int j = 16 * bj + (l & 15);
#pragma unroll 4
        for (int kk = 0; kk < nt16 * 4; ++kk) {
          const int kq = 4 * kk + (l >> 4);
          const double a = Vg[(16 * bi + (l & 15)) * nb + kq];
          const double b = (kq < n && j < n) ? static_cast<double>(Ds[kq * LDD + j]) : 0.0;
          vd[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, vd[q], 0, 0, 0);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MV; ++q) {
      const int t = wv + q * NWV;
      if (t < nt16 * nt16) {
        const int bi = t / nt16, bj = t - (t / nt16) * nt16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * bi + (l >> 4) + 4 * r, j = 16 * bj + (l & 15);
          Vg[i * nb + j] = Vg[i * nb + j] + vd[q][r];
        }
      }
    }
    __syncthreads();
  }

  // SVT weights and P = V diag(w) V^T (exactly symmetric), in storage precision.
  if (tid < n) {
    const double sg = sqrt(fmax(Gp[pk(tid, tid)], 0.0));
    w[tid] = sg > tau ? (sg - tau) / sg : 0.0;
  }
  __syncthreads();
  const gptr<T> Pd = as_global<T>(d.P);
  if constexpr (VG) {
    // upper 16 x 16 blocks of (V diag(w)) V^T on the f64 matrix cores; the
    // f64 result of lane l, register r is entry (l/16 + 4r, l%16); entries
    // with i <= j are written to both halves, so P is exactly symmetric
    typedef double d4 __attribute__((ext_vector_type(4)));
    constexpr int NWV = NT / 64;
    const int wv = tid >> 6, l = tid & 63;
    const int nt16 = nb / 16;
    const int nut = nt16 * (nt16 + 1) / 2;
    for (int t = wv; t < nut; t += NWV) {
      int bj = 0;
      while ((bj + 1) * (bj + 2) / 2 <= t) ++bj;
      const int bi = t - bj * (bj + 1) / 2;
      d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
      for (int kk = 0; kk < nt16 * 4; ++kk) {
        const int kq = 4 * kk + (l >> 4);
        const double a = Vg[(16 * bi + (l & 15)) * nb + kq] * w[kq];
        const double b = Vg[(16 * bj + (l & 15)) * nb + kq];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * bi + (l >> 4) + 4 * r, j = 16 * bj + (l & 15);
        if (i <= j) {
          Pd[i * nb + j] = static_cast<T>(acc[r]);
          Pd[j * nb + i] = static_cast<T>(acc[r]);
        }
      }
    }
  } else {
    const int nbup = nb * (nb + 1) / 2;
    for (int idx = tid; idx < nbup; idx += NT) {
      int j = 0;
      while ((j + 1) * (j + 2) / 2 <= idx) ++j;
      const int i = idx - j * (j + 1) / 2;
      double s = 0.0;
      if (j < n) {
        const double* vi_ = Vs + i * LDV;
        const double* vj_ = Vs + j * LDV;
        s = dot4<NMAX>([&](int k, double acc) { return fma(vi_[k] * w[k], vj_[k], acc); });
      }
      Pd[i * nb + j] = static_cast<T>(s);
      Pd[j * nb + i] = static_cast<T>(s);
    }
    for (int idx = tid; idx < nb * nb; idx += NT) {
      const int i = idx / nb, j = idx - (idx / nb) * nb;
      d.V[idx] = (i < n && j < n) ? Vs[i * LDV + j] : 0.0;
    }
  }
  EIG_MARK(3);
  if (tid == 0) {
    int rank = 0;
    for (int k = 0; k < n; ++k) rank += w[k] != 0.0 ? 1 : 0;
    st->rank = rank;
    st->sweeps = sweeps;
    st->sweeps_total += sweeps;
    st->iter = kd + 1;
  }
#undef EIG_MARK
}

}  // namespace

hipError_t launch_eig_wide(int dtype, int ncls, int grid, hipStream_t stream, const SolveDesc* descs,
                           const int32_t* ids) {
  if (grid <= 0) return hipSuccess;
  const dim3 g(grid), b(kEigWideThreads);
  if (ncls == kEigWideMaxN) {
    if (dtype == 1)
      RPCA_LAUNCH((k_eig_wide<float, kEigWideMaxN, kEigWideThreads>), g, b, 0, stream, descs, ids);
    else
      RPCA_LAUNCH((k_eig_wide<double, kEigWideMaxN, kEigWideThreads>), g, b, 0, stream, descs, ids);
  } else if (ncls == kEigHugeMaxN) {
    if (dtype == 1)
      RPCA_LAUNCH((k_eig_wide<float, kEigHugeMaxN, kEigWideThreads>), g, b, 0, stream, descs, ids);
    else
      RPCA_LAUNCH((k_eig_wide<double, kEigHugeMaxN, kEigWideThreads>), g, b, 0, stream, descs, ids);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace rpca
