// Block-diagonal preconditioner M = S + i dt/2 H0 (eq. matrixM), applied through banded LU factors.
//
// M is block diagonal over channels; each block is factored once per dt (host side, banded LU
// without pivoting: the Hermitian part of M is the SPD overlap S, so no pivot vanishes). Rows are
// ordered q = 2 i + s (radial index, spinor component) so each block is banded with half-width
// w = 2 hb + 1.
//
// The triangular solves are sequential in q. One wave solves one channel; the 2nr rows are split
// into P <= 64 segments of m rows, one per lane:
//   1. every lane substitutes through its segment with a zero boundary window and keeps the
//      last (forward) / first (backward) w values;
//   2. the true boundary windows are propagated segment to segment, t_p = g_p - T_p t_{p-1},
//      with the w x w coupling matrices T_p precomputed at factorisation time (13 lanes, one row
//      of T_p each);
//   3. every lane substitutes through its segment again from its true boundary window.
// Factor storage per block: LU[q][0..w-1] = L(q, q-1-k), LU[q][w] = 1 / U(q, q),
// LU[q][w+1+k] = U(q, q+1+k); TL[p][w][w], TU[p][w][w].
#pragma once
#include "common.hpp"

namespace tdde {

constexpr int kPrecW = 13;        // 2 * hb + 1 for hb = 6 (order-7 B-splines)
constexpr int kPrecStride = 2 * kPrecW + 1;
constexpr int kMaxSeg = 64;

template <typename T> struct DevPrec {
  int n;                   // 2 * nr
  int m;                   // rows per segment (segments 0..P-2 have exactly m rows, m >= w)
  int P;                   // segments
  const int* block_of;     // [nang] factor block of channel j
  const c2_t<T>* LU;       // [nblk][n][kPrecStride]
  const c2_t<T>* TL;       // [nblk][P][w][w]
  const c2_t<T>* TU;       // [nblk][P][w][w]
};

// Vector element of row q in the [s][i] layout of one channel.
__device__ inline size_t prow(int q, int nr) { return (size_t)(q & 1) * nr + (q >> 1); }

// Input of the lower solve, formed on the fly and written back:
//   MODE_P:  z = r + beta (p - omega v)   (BiCGSTAB direction update; z is stored into p)
//   MODE_S:  z = r - alpha v              (BiCGSTAB half step;        z is stored into s)
//   MODE_IN, MODE_IN_S: z = in            (plain preconditioner apply; input not rewritten)
enum { MODE_P = 0, MODE_S = 1, MODE_IN = 2, MODE_FRESH = 3 /* z = r, stored into p */, MODE_IN_S = 4 /* z = s */ };

template <typename T> struct ChainIO {
  const c2_t<T>* r;   // residual (channel base)
  c2_t<T>* pz;        // p or s vector (channel base); input for MODE_IN
  const c2_t<T>* v;   // v (channel base)
  c2_t<T>* out;       // preconditioned result (channel base)
  double2 c1, c2;     // MODE_P: (beta, omega); MODE_S: (alpha, -)
};

// Rows a lane keeps in flight during a substitution: the operands of the next kChainAhead rows are
// loaded before the current row is computed and its results stored, so the loads overlap the
// arithmetic of the rows before them instead of one memory latency being paid per row.
#ifndef TDDE_CHAIN_AHEAD
#define TDDE_CHAIN_AHEAD 2
#endif
constexpr int kChainAhead = TDDE_CHAIN_AHEAD;

// Substitution kinds: lower phase 1 (forms the input), lower phase 3, upper phase 1, upper phase 3.
enum { SUB_L1 = 0, SUB_L3 = 1, SUB_U1 = 2, SUB_U3 = 3 };

// Operands of one row: the factor entries (L row: W values; U row: 1/U(q,q) and W values) and the
// raw vector values the right-hand side is formed from.
template <typename T, int NC> struct RowOps {
  c2_t<T> c[NC];
  c2_t<T> z0, z1, z2;
};

template <typename T, int KIND, int MODE, int NC>
__device__ inline void row_fetch(RowOps<T, NC>& ro, const c2_t<T>* LU, const ChainIO<T>& io, int nr, int q) {
  const size_t e = prow(q, nr);
  const c2_t<T>* row = LU + (size_t)q * kPrecStride + (KIND <= SUB_L3 ? 0 : kPrecW);
#pragma unroll
  for (int k = 0; k < NC; ++k) ro.c[k] = row[k];
  if (KIND == SUB_L1) {
    if constexpr (MODE == MODE_P) { ro.z0 = io.r[e]; ro.z1 = io.pz[e]; ro.z2 = io.v[e]; }
    else if constexpr (MODE == MODE_S) { ro.z0 = io.r[e]; ro.z2 = io.v[e]; }
    else if constexpr (MODE == MODE_FRESH) { ro.z0 = io.r[e]; }
    else { ro.z0 = io.pz[e]; }
  } else if (KIND == SUB_L3) {
    ro.z0 = io.pz[e];  // the input formed (and stored) in phase 1
  } else {
    ro.z0 = io.out[e];  // y of the lower solve (U1), or y overwritten by nothing yet (U3)
  }
}

// Right-hand side value of a lower phase-1 row from its raw operands:
//   MODE_P:  z = r + beta (p - omega v)   (BiCGSTAB direction update; z is stored into p)
//   MODE_S:  z = r - alpha v              (BiCGSTAB half step;        z is stored into s)
//   MODE_FRESH: z = r (stored into p); MODE_IN, MODE_IN_S: z = input (not rewritten)
template <typename T, int MODE, int NC>
__device__ inline c2_t<T> row_input(const RowOps<T, NC>& ro, const ChainIO<T>& io) {
  if constexpr (MODE == MODE_P) {
    const c2_t<T> omega = cmk<T>((T)io.c2.x, (T)io.c2.y), beta = cmk<T>((T)io.c1.x, (T)io.c1.y);
    return cfma<T>(beta, csub<T>(ro.z1, cmul<T>(omega, ro.z2)), ro.z0);
  } else if constexpr (MODE == MODE_S) {
    return csub<T>(ro.z0, cmul<T>(cmk<T>((T)io.c1.x, (T)io.c1.y), ro.z2));
  } else {
    return ro.z0;
  }
}

// One lane's substitution through its segment [o, o+len) from the window win.
//   lower (L1, L3): rows ascending, win[k] = y_{q-1-k}; y_q = z_q - sum_k L(q, q-1-k) win[k]
//   upper (U1, U3): rows descending, win[k] = x_{q+1+k}; x_q = (y_q - sum_k U(q, q+1+k) win[k]) / U(q,q)
// Phase 1 kinds keep only the window (L1 also stores the formed input and accumulates |z|^2);
// phase 3 kinds write the result into io.out.
template <typename T, int KIND, int MODE, int W>
__device__ inline void substitute(const c2_t<T>* LU, const ChainIO<T>& io, int nr, int o, int len, c2_t<T> (&win)[W],
                                  double& nrm2) {
  constexpr bool lower = KIND <= SUB_L3;
  constexpr int NC = lower ? W : W + 1;
  constexpr int D = kChainAhead;
  RowOps<T, NC> ro[D];
#pragma unroll
  for (int d = 0; d < D; ++d)
    if (d < len) row_fetch<T, KIND, MODE, NC>(ro[d], LU, io, nr, lower ? o + d : o + len - 1 - d);
  for (int t0 = 0; t0 < len; t0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int t = t0 + d;
      if (t < len) {
        const int q = lower ? o + t : o + len - 1 - t;
        const size_t e = prow(q, nr);
        c2_t<T> acc;
        if (KIND == SUB_L1) {
          acc = row_input<T, MODE, NC>(ro[d], io);
          nrm2 += (double)acc.x * acc.x + (double)acc.y * acc.y;
        } else {
          acc = ro[d].z0;
        }
        const c2_t<T> zin = acc;
#pragma unroll
        for (int k = 0; k < W; ++k) acc = csub<T>(acc, cmul<T>(ro[d].c[lower ? k : k + 1], win[k]));
        if (!lower) acc = cmul<T>(acc, ro[d].c[0]);
#pragma unroll
        for (int k = W - 1; k > 0; --k) win[k] = win[k - 1];
        win[0] = acc;
        // loads of row t + D are issued before this row's stores, so waiting for them later does
        // not wait for the stores
        if (t + D < len) row_fetch<T, KIND, MODE, NC>(ro[d], LU, io, nr, lower ? o + t + D : o + len - 1 - t - D);
        if (KIND == SUB_L1 && MODE != MODE_IN && MODE != MODE_IN_S) io.pz[e] = zin;
        if (KIND == SUB_L3 || KIND == SUB_U3) io.out[e] = acc;
      }
    }
  }
}

// Ordering of LDS accesses between lanes of one wave: a wave executes its LDS operations in issue
// order, so only the compiler has to be kept from moving them across this point.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Boundary propagation over the segments: lane r < W owns row r of the w x w coupling matrices and
// of the windows; the T row of the next step is loaded one step ahead.
//   lower: t_p = g_p - T_p t_{p-1}, p = 1 .. P-1; upper: h_p = g_p - T_p h_{p+1}, p = P-2 .. 0.
template <typename T, bool LOWER, int W>
__device__ inline void propagate(const c2_t<T>* Tm, int P, c2_t<T>* lds) {
  const int lane = threadIdx.x & 63;
  const int first = LOWER ? 1 : P - 2, count = P - 1;
  c2_t<T> tr[W];
  if (lane < W && count > 0) {
#pragma unroll
    for (int c = 0; c < W; ++c) tr[c] = Tm[((size_t)first * W + lane) * W + c];
  }
  for (int k = 0; k < count; ++k) {
    const int p = LOWER ? first + k : first - k;
    const int prev = LOWER ? p - 1 : p + 1;
    c2_t<T> acc = cmk<T>(0, 0);
    if (lane < W) {
      acc = lds[p * W + lane];
#pragma unroll
      for (int c = 0; c < W; ++c) acc = csub<T>(acc, cmul<T>(tr[c], lds[prev * W + c]));
      if (k + 1 < count) {
        const int pn = LOWER ? p + 1 : p - 1;
#pragma unroll
        for (int c = 0; c < W; ++c) tr[c] = Tm[((size_t)pn * W + lane) * W + c];
      }
    }
    wave_sync();
    if (lane < W) lds[p * W + lane] = acc;
    wave_sync();
  }
}

// Solve M_blk z = input for one channel with one wave (the calling wave; lanes = segments).
// lds: kMaxSeg * W complex values. Returns the |input|^2 sum of the chain (valid in lane 0).
template <typename T, int MODE>
__device__ inline double chain_solve(const DevPrec<T>& pc, int blk, int nr, const ChainIO<T>& io, c2_t<T>* lds) {
  constexpr int W = kPrecW;
  const int lane = threadIdx.x & 63;
  const int P = pc.P, m = pc.m, n = pc.n;
  const c2_t<T>* LU = pc.LU + (size_t)blk * n * kPrecStride;
  const c2_t<T>* TL = pc.TL + (size_t)blk * P * W * W;
  const c2_t<T>* TU = pc.TU + (size_t)blk * P * W * W;
  const int o = lane * m;
  const int len = lane < P ? min(m, n - o) : 0;
  double nrm2 = 0.0, dummy = 0.0;
  c2_t<T> win[W];

  // ---- lower solve, phase 1: local windows; tail t_p[c] = y[o + len - W + c] = win[W-1-c]
#pragma unroll
  for (int k = 0; k < W; ++k) win[k] = cmk<T>(0, 0);
  substitute<T, SUB_L1, MODE, W>(LU, io, nr, o, len, win, nrm2);
  if (lane < P) {
#pragma unroll
    for (int c = 0; c < W; ++c) lds[lane * W + c] = win[W - 1 - c];
  }
  wave_sync();
  // ---- phase 2: true tails
  propagate<T, true, W>(TL, P, lds);
  // ---- phase 3: final substitution from the true window win[k] = y_{o-1-k} = t_{p-1}[W-1-k]
#pragma unroll
  for (int k = 0; k < W; ++k) win[k] = (lane > 0 && lane < P) ? lds[(lane - 1) * W + (W - 1 - k)] : cmk<T>(0, 0);
  wave_sync();
  substitute<T, SUB_L3, MODE, W>(LU, io, nr, o, len, win, dummy);

  // ---- upper solve, phase 1: heads h_p[c] = x[o + c] = win[c] with zero incoming window
#pragma unroll
  for (int k = 0; k < W; ++k) win[k] = cmk<T>(0, 0);
  substitute<T, SUB_U1, MODE, W>(LU, io, nr, o, len, win, dummy);
  if (lane < P) {
#pragma unroll
    for (int c = 0; c < W; ++c) lds[lane * W + c] = win[c];
  }
  wave_sync();
  // ---- phase 2: h_p = g_p - TU_p h_{p+1}, p descending
  propagate<T, false, W>(TU, P, lds);
  // ---- phase 3: x from the true incoming window win[k] = x_{o+len+k} = h_{p+1}[k]
#pragma unroll
  for (int k = 0; k < W; ++k) win[k] = lane + 1 < P ? lds[(lane + 1) * W + k] : cmk<T>(0, 0);
  wave_sync();
  substitute<T, SUB_U3, MODE, W>(LU, io, nr, o, len, win, dummy);
  // |input|^2 of the chain
  for (int off = 32; off > 0; off >>= 1) nrm2 += __shfl_xor(nrm2, off, 64);
  return nrm2;
}

}  // namespace tdde
