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
  int mode;
};

template <typename T>
__device__ inline c2_t<T> chain_input(const ChainIO<T>& io, size_t e, bool store) {
  c2_t<T> z;
  if (io.mode == MODE_P) {
    const c2_t<T> omega = cmk<T>((T)io.c2.x, (T)io.c2.y), beta = cmk<T>((T)io.c1.x, (T)io.c1.y);
    const c2_t<T> pv = csub<T>(io.pz[e], cmul<T>(omega, io.v[e]));
    z = cfma<T>(beta, pv, io.r[e]);
  } else if (io.mode == MODE_S) {
    z = csub<T>(io.r[e], cmul<T>(cmk<T>((T)io.c1.x, (T)io.c1.y), io.v[e]));
  } else if (io.mode == MODE_FRESH) {
    z = io.r[e];
  } else {
    z = io.pz[e];
  }
  if (store && io.mode != MODE_IN && io.mode != MODE_IN_S) io.pz[e] = z;
  return z;
}

// One lane: forward substitution over rows [o, o+len) from the window win (win[k] = y_{o-1-k}).
// phase 1: forms the input (stores it, accumulates |z|^2), keeps the window only.
// phase 3: reads the stored input, writes y into io.out.
template <typename T, int W>
__device__ inline void lower_segment(const c2_t<T>* __restrict__ LU, const ChainIO<T>& io, int nr, int o, int len,
                                     c2_t<T> (&win)[W], bool phase1, double& nrm2) {
  for (int q = o; q < o + len; ++q) {
    const size_t e = prow(q, nr);
    c2_t<T> acc;
    if (phase1) {
      acc = chain_input<T>(io, e, true);
      nrm2 += (double)acc.x * acc.x + (double)acc.y * acc.y;
    } else {
      acc = io.pz[e];  // the input formed (and stored) in phase 1
    }
    const c2_t<T>* row = LU + (size_t)q * kPrecStride;
#pragma unroll
    for (int k = 0; k < W; ++k) acc = csub<T>(acc, cmul<T>(row[k], win[k]));
#pragma unroll
    for (int k = W - 1; k > 0; --k) win[k] = win[k - 1];
    win[0] = acc;
    if (!phase1) io.out[e] = acc;
  }
}

// One lane: backward substitution over rows [o, o+len) (q descending) from the window
// win (win[k] = x_{o+len+k}). Reads y from io.out; phase 3 overwrites it with x.
template <typename T, int W>
__device__ inline void upper_segment(const c2_t<T>* __restrict__ LU, const ChainIO<T>& io, int nr, int o, int len,
                                     c2_t<T> (&win)[W], bool phase1) {
  for (int q = o + len - 1; q >= o; --q) {
    const size_t e = prow(q, nr);
    c2_t<T> acc = io.out[e];
    const c2_t<T>* row = LU + (size_t)q * kPrecStride;
#pragma unroll
    for (int k = 0; k < W; ++k) acc = csub<T>(acc, cmul<T>(row[W + 1 + k], win[k]));
    acc = cmul<T>(acc, row[W]);
#pragma unroll
    for (int k = W - 1; k > 0; --k) win[k] = win[k - 1];
    win[0] = acc;
    if (!phase1) io.out[e] = acc;
  }
}

// Solve M_blk z = input for one channel with one wave (the calling wave; lanes = segments).
// lds: kMaxSeg * W complex values. Returns the |input|^2 sum of the chain (valid in lane 0).
template <typename T>
__device__ inline double chain_solve(const DevPrec<T>& pc, int blk, int nr, const ChainIO<T>& io, c2_t<T>* lds) {
  constexpr int W = kPrecW;
  const int lane = threadIdx.x & 63;
  const int P = pc.P, m = pc.m, n = pc.n;
  const c2_t<T>* LU = pc.LU + (size_t)blk * n * kPrecStride;
  const c2_t<T>* TL = pc.TL + (size_t)blk * P * W * W;
  const c2_t<T>* TU = pc.TU + (size_t)blk * P * W * W;
  const int o = lane * m;
  const int len = lane < P ? min(m, n - o) : 0;
  double nrm2 = 0.0;
  c2_t<T> win[W];

  // ---- lower solve, phase 1: local windows
#pragma unroll
  for (int k = 0; k < W; ++k) win[k] = cmk<T>(0, 0);
  if (len > 0) lower_segment<T, W>(LU, io, nr, o, len, win, true, nrm2);
  // tail t_p[c] = y[o + len - W + c] = win[W-1-c]
  if (lane < P) {
#pragma unroll
    for (int c = 0; c < W; ++c) lds[lane * W + c] = win[W - 1 - c];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  // ---- phase 2: t_p = g_p - T_p t_{p-1}, sequential over p, lanes 0..W-1 own rows of T_p
  for (int p = 1; p < P; ++p) {
    c2_t<T> acc = cmk<T>(0, 0);
    if (lane < W) {
      acc = lds[p * W + lane];
      const c2_t<T>* Tp = TL + ((size_t)p * W + lane) * W;
#pragma unroll
      for (int c = 0; c < W; ++c) acc = csub<T>(acc, cmul<T>(Tp[c], lds[(p - 1) * W + c]));
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    if (lane < W) lds[p * W + lane] = acc;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
  // ---- phase 3: final substitution from the true window win[k] = y_{o-1-k} = t_{p-1}[W-1-k]
  if (len > 0) {
#pragma unroll
    for (int k = 0; k < W; ++k) win[k] = lane > 0 ? lds[(lane - 1) * W + (W - 1 - k)] : cmk<T>(0, 0);
    double dummy = 0.0;
    lower_segment<T, W>(LU, io, nr, o, len, win, false, dummy);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");

  // ---- upper solve, phase 1: heads h_p[c] = x[o + c] = win[c] with zero incoming window
#pragma unroll
  for (int k = 0; k < W; ++k) win[k] = cmk<T>(0, 0);
  if (len > 0) upper_segment<T, W>(LU, io, nr, o, len, win, true);
  if (lane < P) {
#pragma unroll
    for (int c = 0; c < W; ++c) lds[lane * W + c] = win[c];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  // ---- phase 2: h_p = g_p - TU_p h_{p+1}, p descending
  for (int p = P - 2; p >= 0; --p) {
    c2_t<T> acc = cmk<T>(0, 0);
    if (lane < W) {
      acc = lds[p * W + lane];
      const c2_t<T>* Tp = TU + ((size_t)p * W + lane) * W;
#pragma unroll
      for (int c = 0; c < W; ++c) acc = csub<T>(acc, cmul<T>(Tp[c], lds[(p + 1) * W + c]));
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    if (lane < W) lds[p * W + lane] = acc;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
  // ---- phase 3: x from the true incoming window win[k] = x_{o+len+k} = h_{p+1}[k]
  if (len > 0) {
#pragma unroll
    for (int k = 0; k < W; ++k) win[k] = lane + 1 < P ? lds[(lane + 1) * W + k] : cmk<T>(0, 0);
    upper_segment<T, W>(LU, io, nr, o, len, win, false);
  }
  // |input|^2 of the chain
  for (int off = 32; off > 0; off >>= 1) nrm2 += __shfl_xor(nrm2, off, 64);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  return nrm2;
}

}  // namespace tdde
