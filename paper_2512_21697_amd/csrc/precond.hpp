// Block-diagonal preconditioner M = S + i dt/2 H0 (eq. matrixM), applied through banded LU factors.
//
// M is block diagonal over channels; each block is factored once per dt (host side, banded LU
// without pivoting: the Hermitian part of M is the SPD overlap S, so no pivot vanishes). Rows are
// ordered q = 2 i + s (radial index, spinor component) so each block is banded with half-width
// w = 2 hb + 1.
//
// The triangular solves are sequential in q. One work-group solves one channel; the 2nr rows are
// split into P <= 256 segments of m >= w rows, one per thread:
//   1. every thread substitutes through its segment with a zero boundary window and keeps the
//      last (forward) / first (backward) w values;
//   2. the true boundary windows follow from t_p = g_p - T_p t_{p-1} (w x w coupling matrices T_p
//      precomputed at factorisation time), in two levels: within groups of kSegGroup segments
//      (13 threads per group, groups in parallel, started from a zero window), then across the
//      group boundaries with the precomputed group products C_p, and finally every window is
//      corrected by C_p times the true boundary entering its group;
//   3. every thread substitutes through its segment again from its true boundary window.
// A work-group solves nc channels of one factor block at once (nc = 256 / P rounded down to a power of
// two, at most 8): lane t = p nc + kk runs segment p of channel kk, so the nc lanes that read the same
// factor rows sit side by side in one wave and every factor load of a wave touches the rows of 64 / nc
// segments once; phase 2 runs for all channels side by side (kSegGroup-segment groups of every
// channel in their own slots; boundary windows in LDS by channel, win[kk P + p]).
// Factor storage per block, row q = p m + t of segment p: entry k of the row is LU[t][k][p] (the
// segment index fastest, so the threads of a wave read consecutive addresses), with entries
// 0..w-1 = L(q, q-1-k), w = 1 / U(q, q), w+1+k = U(q, q+1+k); TL, TU [p][c][r] = T_p(r, c);
// CL, CU [r][c][p].
#pragma once
#include "common.hpp"

namespace tdde {

constexpr int kPrecW = 13;        // 2 * hb + 1 for hb = 6 (order-7 B-splines)
constexpr int kPrecStride = 2 * kPrecW + 1;
constexpr int kMaxSeg = kThreads;   // one segment per thread of the work-group
constexpr int kSegGroup = 16;       // segments per group of the two-level boundary propagation
constexpr int kMaxSegGroups = kMaxSeg / kSegGroup;

template <typename T> struct DevPrec {
  int n;                   // 2 * nr
  int m;                   // rows per segment (segments 0..P-2 have exactly m rows, m >= w)
  int P;                   // segments
  const int* block_of;     // [nang] factor block of channel j
  int nc;                  // channels of one block solved together by a work-group (1, 2, 4 or 8)
  const int* chain_order;  // [n_items][nc] channels of chain work item w (-1: none), see chain_order_of
  int n_items;
  const c2_t<T>* LU;       // [nblk][m][kPrecStride][P]: entry k of row t of segment p
  const c2_t<T>* TL;       // [nblk][P][w][w] transposed per segment: TL[p][c][r] = T_p(r, c)
  const c2_t<T>* TU;       // [nblk][P][w][w] likewise
  const c2_t<T>* CL;       // [nblk][w][w][P] lower group products
  const c2_t<T>* CU;       // [nblk][w][w][P] upper group products
};

// Steps of every segment staged through LDS at a time in the substitutions, at most (one staging
// round trip per chunk: 16 is the most that keeps two chain work-groups per CU; segments whose length
// is not a multiple of 16 take chunks of 8, see substitute_chunked), and the row pitch of the staging
// array (kMaxSeg + 2: the cooperative writes of one segment's consecutive steps by 16 lanes hit 16
// different 16-byte bank groups).
constexpr int kStageRows = 16;
constexpr int kStagePitch = kMaxSeg + 2;

// LDS of one chain solve: the boundary window of every segment and the true boundary of every
// segment group (phase 2); the staged steps of the substitutions share the windows' space.
constexpr int kMaxChainNc = 8;  // channels of one work-group

template <typename T> struct ChainLds {
  union {
    c2_t<T> win[kMaxSeg][kPrecW];
    c2_t<T> stage[kStageRows][kStagePitch];
  };
  c2_t<T> u[kMaxSegGroups][kPrecW];
  long coff[kMaxChainNc];  // element offset of every channel of the work item within the instance
};
static_assert(sizeof(ChainLds<double>) <= 80 * 1024, "two chain work-groups per CU");

// Channels of chain work item w (pc.chain_order row): count of valid entries (0 for a padding item).
template <typename T> __device__ inline int chain_item(const DevPrec<T>& pc, int w, const int*& js) {
  js = pc.chain_order + (size_t)w * pc.nc;
  int nk = 0;
  while (nk < pc.nc && js[nk] >= 0) ++nk;
  return nk;
}

// Vector element of row q in the [s][i] layout of one channel.
__device__ inline size_t prow(int q, int nr) { return (size_t)(q & 1) * nr + (q >> 1); }

// Input of the lower solve, formed on the fly and written back:
//   MODE_P:  z = r + beta (p - omega v)   (BiCGSTAB direction update; z is stored into p)
//   MODE_S:  z = r - alpha v              (BiCGSTAB half step;        z is stored into s)
//   MODE_IN, MODE_IN_S: z = in            (plain preconditioner apply; input not rewritten)
enum { MODE_P = 0, MODE_S = 1, MODE_IN = 2, MODE_FRESH = 3 /* z = r, stored into p */, MODE_IN_S = 4 /* z = s */ };

template <typename T> struct ChainIO {
  const c2_t<T>* r;   // residual (instance base)
  c2_t<T>* pz;        // p or s vector (instance base); input for MODE_IN
  const c2_t<T>* v;   // v (instance base)
  c2_t<T>* out;       // preconditioned result (instance base)
  double2 c1, c2;     // MODE_P: (beta, omega); MODE_S: (alpha, -)
};

// Rows of factor operands a lane keeps in flight during a substitution: the factors of the next
// kChainAhead rows are loaded before the current row is computed.
#ifndef TDDE_CHAIN_AHEAD
#define TDDE_CHAIN_AHEAD 1
#endif
constexpr int kChainAhead = TDDE_CHAIN_AHEAD;


// Substitution kinds: lower phase 1 (forms the input), lower phase 3, upper phase 1, upper phase 3.
enum { SUB_L1 = 0, SUB_L3 = 1, SUB_U1 = 2, SUB_U3 = 3 };

// Complex value of another precision (the factors may be stored in FP32 for an FP64 solve).
template <typename T> __device__ inline c2_t<T> cvt(double2 z) { return cmk<T>((T)z.x, (T)z.y); }
template <typename T> __device__ inline c2_t<T> cvt(float2 z) { return cmk<T>((T)z.x, (T)z.y); }

// Factor entries of one row: L row: W values; U row: 1/U(q,q) and W values.
template <typename T, int NC> struct RowOps {
  c2_t<T> c[NC];
};

// LU: the block's factors offset to the calling thread's segment (entry stride P); t: row of the segment.
template <typename T, int KIND, int NC>
__device__ inline void row_fetch(RowOps<T, NC>& ro, const c2_t<T>* LU, int t, int P) {
  const c2_t<T>* row = LU + ((size_t)t * kPrecStride + (KIND <= SUB_L3 ? 0 : kPrecW)) * P;
#pragma unroll
  for (int k = 0; k < NC; ++k) ro.c[k] = gld(row + (size_t)k * P);
}

// Vector element of step u of segment p in a pass (lower passes walk rows o + u upwards, upper
// passes rows o + len - 1 - u downwards), or -1 past the segment's rows.
__device__ inline long step_elem(int p, int u, int m, int n, int nr, bool lower) {
  const int o = p * m;
  const int len = min(m, n - o);
  if (u >= len) return -1;
  return (long)prow(lower ? o + u : o + len - 1 - u, nr);
}

// Input of one row of a pass at vector element e, loaded by the cooperative staging:
//   L1: MODE_P z = r + beta (p - omega v) (stored into p), MODE_S z = r - alpha v (stored into s),
//       MODE_FRESH z = r (stored into p), MODE_IN / MODE_IN_S z = the input (not rewritten);
//   L3: z again; U1, U3: y of the lower solve (in out).
template <typename T, int KIND, int MODE>
__device__ inline c2_t<T> stage_input(const ChainIO<T>& io, long e) {
  if constexpr (KIND == SUB_L1) {
    if constexpr (MODE == MODE_P) {
      const c2_t<T> omega = cmk<T>((T)io.c2.x, (T)io.c2.y), beta = cmk<T>((T)io.c1.x, (T)io.c1.y);
      const c2_t<T> z = cfma<T>(beta, csub<T>(gld(io.pz + e), cmul<T>(omega, gld(io.v + e))), gld(io.r + e));
      gst(io.pz + e, z);
      return z;
    } else if constexpr (MODE == MODE_S) {
      const c2_t<T> z = csub<T>(gld(io.r + e), cmul<T>(cmk<T>((T)io.c1.x, (T)io.c1.y), gld(io.v + e)));
      gst(io.pz + e, z);
      return z;
    } else if constexpr (MODE == MODE_FRESH) {
      const c2_t<T> z = gld(io.r + e);
      gst(io.pz + e, z);
      return z;
    } else {
      return gld(io.pz + e);
    }
  } else if constexpr (KIND == SUB_L3) {
    return gld(io.pz + e);
  } else {
    return gld(io.out + e);
  }
}

// One pass of substitutions, every lane through its segment (len rows) from the window win:
//   lower (L1, L3): rows ascending, win[k] = y_{q-1-k}; y_q = z_q - sum_k L(q, q-1-k) win[k]
//   upper (U1, U3): rows descending, win[k] = x_{q+1+k}; x_q = (y_q - sum_k U(q, q+1+k) win[k]) / U(q,q)
// The pass runs in chunks of kStageRows steps of every segment of the nk channels: the work-group
// loads the chunk's inputs into LDS (consecutive threads take consecutive rows of one segment, so a
// wave's loads are runs of whole pieces instead of one element per segment m / 2 elements apart),
// every lane substitutes its rows from LDS, and phase-3 kinds write their results back through LDS
// the same way. Phase-1 kinds keep only the window. All threads call (barriers inside).
template <typename T, int KIND, int MODE, int W, int D, typename TF, int C>
__device__ inline void substitute(const c2_t<TF>* LU, int P, int m, int n, int nc, int nk, const ChainIO<T>& io, int nr,
                                  int len, c2_t<T> (&win)[W], ChainLds<T>& L) {
  constexpr bool lower = KIND <= SUB_L3;
  constexpr bool writes = KIND == SUB_L3 || KIND == SUB_U3;
  constexpr int NC = lower ? W : W + 1;
  static_assert(C <= kStageRows, "chunk larger than the staging array");
  static_assert(C % D == 0, "the steps of a chunk must be whole rounds of the lookahead");
  const int lane = threadIdx.x;
  const int nl = nc * P;  // lanes that may hold a segment (those of channel slots kk >= nk hold none)
  RowOps<TF, NC> ro[D];
#pragma unroll
  for (int d = 0; d < D; ++d)
    if (d < len) row_fetch<TF, KIND, NC>(ro[d], LU, lower ? d : len - 1 - d, P);
  auto elem = [&](int idx, int c0, int& uu) {
    const int ln = idx / C;
    uu = idx - ln * C;
    const int kk = ln % nc;
    if (kk >= nk) return -1L;
    const long e = step_elem(ln / nc, c0 + uu, m, n, nr, lower);
    return e >= 0 ? L.coff[kk] + e : -1L;
  };
  for (int c0 = 0; c0 < m; c0 += C) {
    __syncthreads();  // the previous chunk (or the caller's use of this LDS) is finished
    for (int idx = threadIdx.x; idx < nl * C; idx += kThreads) {
      int uu;
      const long e = elem(idx, c0, uu);
      if (e >= 0) L.stage[uu][idx / C] = stage_input<T, KIND, MODE>(io, e);
    }
    __syncthreads();
    for (int u0 = 0; u0 < C; u0 += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int uu = u0 + d, u = c0 + uu;
        if (u < len) {
          c2_t<T> acc = L.stage[uu][lane];
#pragma unroll
          for (int k = 0; k < W; ++k) acc = cfms<T>(cvt<T>(ro[d].c[lower ? k : k + 1]), win[k], acc);
          if (!lower) acc = cmul<T>(acc, cvt<T>(ro[d].c[0]));
#pragma unroll
          for (int k = W - 1; k > 0; --k) win[k] = win[k - 1];
          win[0] = acc;
          if (u + D < len) row_fetch<TF, KIND, NC>(ro[d], LU, lower ? u + D : len - 1 - u - D, P);
          if (writes) L.stage[uu][lane] = acc;
        }
      }
    }
    if (writes) {
      __syncthreads();
      for (int idx = threadIdx.x; idx < nl * C; idx += kThreads) {
        int uu;
        const long e = elem(idx, c0, uu);
        if (e >= 0) gst(io.out + e, L.stage[uu][idx / C]);
      }
    }
  }
}

// The substitution in chunks of 16 steps when the segment length is a multiple of 16, else of 8 (a
// 16-step chunk over 24-row segments leaves half of every second chunk empty: the hydrogen step
// measured 2-7 % slower with it, the 64-row beyond-dipole step 1.4 % faster).
template <typename T, int KIND, int MODE, int W, int D = kChainAhead, typename TF = T>
__device__ inline void substitute_chunked(const c2_t<TF>* LU, int P, int m, int n, int nc, int nk,
                                          const ChainIO<T>& io, int nr, int len, c2_t<T> (&win)[W], ChainLds<T>& L) {
  if (m % 16 == 0) substitute<T, KIND, MODE, W, D, TF, 16>(LU, P, m, n, nc, nk, io, nr, len, win, L);
  else substitute<T, KIND, MODE, W, D, TF, 8>(LU, P, m, n, nc, nk, io, nr, len, win, L);
}

// Ordering of LDS accesses between lanes of one wave: a wave executes its LDS operations in issue
// order, so only the compiler has to be kept from moving them across this point.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Phase 2, first level: the recurrence inside every group of kSegGroup segments of every channel,
// started from the group's own zero-window tail. Channel kk's groups occupy slots kk * GS .. kk * GS +
// GS - 1 (GS = kMaxSegGroups / nc); wave v owns slots 4v .. 4v+3 and lane 13 k + r (k < 4) row r of
// slot 4v + k. The T row of the next step is loaded one step ahead.
//   lower: t_p = g_p - T_p t_{p-1}, p ascending from the group's first segment;
//   upper: h_p = g_p - T_p h_{p+1}, p descending from the group's last segment.
template <typename T, bool LOWER, int W, typename TF = T>
__device__ inline void group_recurrence(const c2_t<TF>* Tm, int P, int nc, int nk, ChainLds<T>& L) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int k = lane / W, r = lane - k * W;
  const int slot = wave * 4 + k, GS = kMaxSegGroups / nc;
  const int kk = slot / GS, g = slot - kk * GS;
  const int lo = g * kSegGroup, hi = min(lo + kSegGroup - 1, P - 1);
  const bool act = lane < 4 * W && kk < nk && lo < P;
  const int base = kk * P;  // lane of the channel's segment 0
  c2_t<TF> tr[W];
  auto fetch = [&](int step) {
    const int p = LOWER ? lo + step : hi - step;
    if (act && step < kSegGroup && (LOWER ? p <= hi : p >= lo)) {
#pragma unroll
      for (int c = 0; c < W; ++c) tr[c] = gld(Tm + ((size_t)p * W + c) * W + r);
    }
  };
  fetch(1);
  for (int step = 1; step < kSegGroup; ++step) {
    const int p = LOWER ? lo + step : hi - step;
    const bool on = act && (LOWER ? p <= hi : p >= lo);
    c2_t<T> acc = cmk<T>(0, 0);
    if (on) {
      const int prev = LOWER ? p - 1 : p + 1;
      acc = L.win[base + p][r];
#pragma unroll
      for (int c = 0; c < W; ++c) acc = cfms<T>(cvt<T>(tr[c]), L.win[base + prev][c], acc);
    }
    fetch(step + 1);
    wave_sync();
    if (on) L.win[base + p][r] = acc;
    wave_sync();
  }
}

// Phase 2, second level (16 threads per channel, rows r < W, channel kk = thread / 16): the true
// boundary of every group of the channel, in order,
//   lower: u_0 = t_hi(0), u_G = t^loc_hi(G) + CL_hi(G) u_{G-1};
//   upper: u_last = h_lo(last), u_G = h^loc_lo(G) + CU_lo(G) u_{G+1}.
template <typename T, bool LOWER, int W, typename TF = T>
__device__ inline void group_boundaries(const c2_t<TF>* Cm, int P, int nc, int nk, ChainLds<T>& L) {
  const int kk = threadIdx.x >> 4, r = threadIdx.x & 15;
  if (kk >= nk || r >= W) return;
  const int NG = (P + kSegGroup - 1) / kSegGroup;
  const int base = kk * P, us = kk * (kMaxSegGroups / nc);  // channel's first lane, first group slot
  const size_t cs = (size_t)P;  // stride between (row, column) planes of C
  auto seg_of = [&](int G) { return LOWER ? min(G * kSegGroup + kSegGroup - 1, P - 1) : G * kSegGroup; };
  const int G0 = LOWER ? 0 : NG - 1;
  L.u[us + G0][r] = L.win[base + seg_of(G0)][r];
  c2_t<TF> cr[W];
  auto fetch = [&](int G) {
    if (G >= 0 && G < NG && G != G0) {
      const int p = seg_of(G);
#pragma unroll
      for (int c = 0; c < W; ++c) cr[c] = gld(Cm + ((size_t)r * W + c) * cs + p);
    }
  };
  fetch(LOWER ? 1 : NG - 2);
  for (int step = 1; step < NG; ++step) {
    const int G = LOWER ? step : NG - 1 - step;
    const int Gin = LOWER ? G - 1 : G + 1;
    wave_sync();
    c2_t<T> acc = L.win[base + seg_of(G)][r];
#pragma unroll
    for (int c = 0; c < W; ++c) acc = cadd<T>(acc, cmul<T>(cvt<T>(cr[c]), L.u[us + Gin][c]));
    fetch(LOWER ? G + 1 : G - 1);
    wave_sync();
    L.u[us + G][r] = acc;
  }
}

// True boundary window of segment q of channel kk into out[W]: the group-local window corrected by
// the group product times the true boundary entering the group (nothing to correct in the group where
// the recurrence starts).
template <typename T, bool LOWER, int W, typename TF = T>
__device__ inline void true_window(const c2_t<TF>* Cm, int P, int nc, int kk, int q, const ChainLds<T>& L,
                                   c2_t<T> (&out)[W]) {
  const int NG = (P + kSegGroup - 1) / kSegGroup;
  const int G = q / kSegGroup;
#pragma unroll
  for (int c = 0; c < W; ++c) out[c] = L.win[kk * P + q][c];
  const bool corr = LOWER ? G > 0 : G < NG - 1;
  if (corr) {
    const c2_t<T>* ub = L.u[kk * (kMaxSegGroups / nc) + (LOWER ? G - 1 : G + 1)];
    c2_t<T> uu[W];
#pragma unroll
    for (int c = 0; c < W; ++c) uu[c] = ub[c];
#pragma unroll
    for (int rr = 0; rr < W; ++rr) {
      c2_t<T> acc = out[rr];
#pragma unroll
      for (int c = 0; c < W; ++c) acc = cadd<T>(acc, cmul<T>(cvt<T>(gld(Cm + ((size_t)rr * W + c) * P + q)), uu[c]));
      out[rr] = acc;
    }
  }
}

// Solve M_blk z = input for the channels js[0 .. nk) (nk <= pc.nc) of factor block blk with the whole
// work-group (all threads call it). io holds the instance's vectors; D: rows of factor operands a lane
// keeps in flight in the substitutions.
template <typename T, int MODE, int D = kChainAhead, typename TF = T>
__device__ __attribute__((noinline)) void chain_solve(const DevPrec<TF>& pc, int blk, int nr, const ChainIO<T>& io,
                                                      const int* js, int nk, ChainLds<T>& L) {
  constexpr int W = kPrecW;
  const int t = threadIdx.x;
  const int P = pc.P, m = pc.m, n = pc.n, nc = pc.nc;
  const int kk = t % nc, p = t / nc;  // channel slot and segment of this lane
  const bool on = kk < nk && p < P;
  const c2_t<TF>* LU = pc.LU + (size_t)blk * m * kPrecStride * P + (on ? p : 0);
  const size_t tsz = (size_t)P * W * W;
  const c2_t<TF>* TL = pc.TL + blk * tsz;
  const c2_t<TF>* TU = pc.TU + blk * tsz;
  const c2_t<TF>* CL = pc.CL + blk * tsz;
  const c2_t<TF>* CU = pc.CU + blk * tsz;
  const int len = on ? min(m, n - p * m) : 0;
  c2_t<T> win[W], tw[W];
  __syncthreads();  // a previous solve of this work-group has finished with coff
  if (t < nk) L.coff[t] = (long)js[t] * 2 * nr;  // read after the first substitution's barrier

  // ---- lower solve, phase 1: local windows; tail t_p[c] = y[o + len - W + c] = win[W-1-c]
#pragma unroll
  for (int k = 0; k < W; ++k) win[k] = cmk<T>(0, 0);
  substitute_chunked<T, SUB_L1, MODE, W, D, TF>(LU, P, m, n, nc, nk, io, nr, len, win, L);
  __syncthreads();  // every lane is done with the staged steps
  if (on) {
#pragma unroll
    for (int c = 0; c < W; ++c) L.win[kk * P + p][c] = win[W - 1 - c];
  }
  __syncthreads();
  // ---- phase 2: group recurrences, group boundaries
  group_recurrence<T, true, W, TF>(TL, P, nc, nk, L);
  __syncthreads();
  group_boundaries<T, true, W, TF>(CL, P, nc, nk, L);
  __syncthreads();
  // ---- phase 3: final substitution from the true window win[k] = y_{o-1-k} = t_{p-1}[W-1-k]
  if (on && p > 0) {
    true_window<T, true, W, TF>(CL, P, nc, kk, p - 1, L, tw);
#pragma unroll
    for (int k = 0; k < W; ++k) win[k] = tw[W - 1 - k];
  } else {
#pragma unroll
    for (int k = 0; k < W; ++k) win[k] = cmk<T>(0, 0);
  }
  substitute_chunked<T, SUB_L3, MODE, W, D, TF>(LU, P, m, n, nc, nk, io, nr, len, win, L);

  // ---- upper solve, phase 1: heads h_p[c] = x[o + c] = win[c] with zero incoming window
#pragma unroll
  for (int k = 0; k < W; ++k) win[k] = cmk<T>(0, 0);
  substitute_chunked<T, SUB_U1, MODE, W, D, TF>(LU, P, m, n, nc, nk, io, nr, len, win, L);
  __syncthreads();  // every thread has read its lower window
  if (on) {
#pragma unroll
    for (int c = 0; c < W; ++c) L.win[kk * P + p][c] = win[c];
  }
  __syncthreads();
  group_recurrence<T, false, W, TF>(TU, P, nc, nk, L);
  __syncthreads();
  group_boundaries<T, false, W, TF>(CU, P, nc, nk, L);
  __syncthreads();
  // ---- phase 3: x from the true incoming window win[k] = x_{o+len+k} = h_{p+1}[k]
  if (on && p + 1 < P) {
    true_window<T, false, W, TF>(CU, P, nc, kk, p + 1, L, tw);
#pragma unroll
    for (int k = 0; k < W; ++k) win[k] = tw[k];
  } else {
#pragma unroll
    for (int k = 0; k < W; ++k) win[k] = cmk<T>(0, 0);
  }
  substitute_chunked<T, SUB_U3, MODE, W, D, TF>(LU, P, m, n, nc, nk, io, nr, len, win, L);
}

}  // namespace tdde
