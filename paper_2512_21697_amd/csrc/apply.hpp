// Matrix-free apply of S and H(t) on one (instance, channel, radial tile) of x[b][j][s][i].
//
// eq. fullH: (H x)[j][s][i] = sum_{s',d} H0_j[s][s'][d][i] x[j][s'][i+d]
//                           + sum_m coef_m f_m sum_{j'} (K^a A_m K^b)[j][j'] sum_{s',d} R_m[s][s'][d][i] x[j'][s'][i+d]
// with H0_j = sum_n kappa_j^n h_n (+ per-channel complex band), S_j = sum_n kappa_j^n s_n or I; the
// kappa polynomials are summed once per distinct kappa on the host, so a tap is one band load.
//
// Work-group layout: 256 threads = 2 components x kStage staged radial points. Thread (s, k) stages
// x[j][s][i0 - hb + k] and, for every term of a pattern group (terms sharing the union of their
// angular sparsity patterns), the angular combination w_m = sum_j' A_m[j][j'] x[j'] at that point:
// all neighbour loads of its point are issued together, each neighbouring value is loaded once for
// all terms of the group. Thread (s, k) with hb <= k < kStage - hb owns y[j][s][i0 - hb + k]; its
// radial band contractions read the staged values from LDS.
#pragma once
#include "common.hpp"

namespace tdde {

constexpr int kGatherMax = 64;    // CSR entries of one pattern row staged in LDS at a time
constexpr int kGatherBatch = 20;  // neighbour loads of a gather issued together (a whole row of the
                                  // |dl| <= 2, mu' = mu +- 1 pattern: at most 20 entries)

template <typename T> struct TileLds {
  c2_t<T> xs[2][kStage];
  c2_t<T> ws[kMaxGroup][2][kStage];
  int gcol[kGatherMax];
  T gval[kGatherMax * kMaxGroup];
};

// Coupling-term table of one instance at one time, in LDS: coef_f[m] = coef_m * f_{field_m}(t);
// per group slot the term index and its nonzero-block mask; g_live[g] when any coefficient of
// group g is nonzero.
struct TermLds {
  double2 coef_f[kMaxTerms];
  int g_first[kMaxTerms + 1];
  int g_term[kMaxTerms];
  int g_mask[kMaxTerms];
  int g_live[kMaxTerms];
};

// Constant part of the term table: the group layout (all threads call; ends with a barrier).
template <typename T>
__device__ inline void terms_layout(const DevOp<T>& op, TermLds& tl) {
  __syncthreads();
  const int t = threadIdx.x;
  if (t < op.n_terms) {
    const int m = op.g_term[t];
    tl.g_term[t] = m;
    tl.g_mask[t] = op.t_mask[m];
  }
  if (t <= op.n_groups) tl.g_first[t] = op.g_first[t];
  __syncthreads();
}

// Time-dependent part: coef_f[m] = cf(m) for the calling thread's term m = threadIdx.x, and the
// group liveness (all threads call; ends with a barrier).
template <typename F>
__device__ inline void terms_fields(int n_terms, int n_groups, TermLds& tl, F&& cf) {
  __syncthreads();
  const int t = threadIdx.x;
  if (t < n_terms) tl.coef_f[t] = cf(t);
  __syncthreads();
  if (t < n_groups) {
    bool any = false;
    for (int q = tl.g_first[t]; q < tl.g_first[t + 1]; ++q) {
      const double2 c = tl.coef_f[tl.g_term[q]];
      any = any || c.x != 0.0 || c.y != 0.0;
    }
    tl.g_live[t] = any ? 1 : 0;
  }
  __syncthreads();
}

// Whole table at once. fval(m) = f_{field_m}(t).
template <typename T, typename F>
__device__ inline void terms_to_lds(const DevOp<T>& op, TermLds& tl, F&& fval) {
  terms_layout<T>(op, tl);
  terms_fields(op.n_terms, op.n_groups, tl, [&](int m) {
    const double f = fval(m);
    const double2 c = op.t_coef[m];
    return make_double2(c.x * f, c.y * f);
  });
}

// Entries [p0, p1) of one pattern-group CSR row (column indices and the K term values of every
// entry; p1 - p0 <= kGatherMax) into LDS. val points at the values of entry p0.
template <typename T>
__device__ inline void stage_csr(TileLds<T>& L, const int* __restrict__ col, const T* __restrict__ val, int p0, int p1,
                                 int K) {
  const int n = p1 - p0;
  for (int k = threadIdx.x; k < n; k += kThreads) L.gcol[k] = col[p0 + k];
  for (int k = threadIdx.x; k < n * K; k += kThreads) L.gval[k] = val[k];
}

// Angular combinations acc_q += sum_p gval[p * K + q] x[gcol[p]][s][ic] of the K terms of one
// pattern group at the calling thread's staged point, over the n <= kGatherMax CSR entries staged in
// LDS (stage_csr). The neighbour loads of GB entries are issued together before any is used (GB at
// least the row length: one memory round trip for the whole gather); column indices and values come
// from LDS only, so no neighbour load waits for another.
template <typename T> struct GatherAcc { c2_t<T> v[kMaxGroup]; };

template <typename T, int GB, int KC>
__device__ __attribute__((always_inline)) inline void gather_fma(const TileLds<T>& L, const c2_t<T> (&xv)[GB], int pb,
                                                                 int n, GatherAcc<T>& acc) {
#pragma unroll
  for (int u = 0; u < GB; ++u) {
    if (pb + u < n) {  // uniform
      const T* v = L.gval + (pb + u) * KC;
      T c[KC];
#pragma unroll
      for (int q = 0; q < KC; ++q) c[q] = v[q];
#pragma unroll
      for (int q = 0; q < KC; ++q) acc.v[q] = rfma<T>(c[q], xv[u], acc.v[q]);
    }
  }
}

template <typename T, int GB>
__device__ __attribute__((always_inline)) inline void gather_point(const TileLds<T>& L,
                                                                   const c2_t<T>* __restrict__ xcol0, int n, int K,
                                                                   size_t cstride, GatherAcc<T>& acc) {
  for (int pb = 0; pb < n; pb += GB) {
    c2_t<T> xv[GB];
#pragma unroll
    for (int u = 0; u < GB; ++u) {
      xv[u] = cmk<T>(0, 0);
      if (pb + u < n) xv[u] = xcol0[(size_t)L.gcol[pb + u] * cstride];  // n uniform: scalar branch
    }
    // the multiply-adds with the group size as a compile-time constant (branch-free inner loop)
    switch (K) {
      case 1: gather_fma<T, GB, 1>(L, xv, pb, n, acc); break;
      case 2: gather_fma<T, GB, 2>(L, xv, pb, n, acc); break;
      case 3: gather_fma<T, GB, 3>(L, xv, pb, n, acc); break;
      case 4: gather_fma<T, GB, 4>(L, xv, pb, n, acc); break;
      case 5: gather_fma<T, GB, 5>(L, xv, pb, n, acc); break;
      case 6: gather_fma<T, GB, 6>(L, xv, pb, n, acc); break;
      case 7: gather_fma<T, GB, 7>(L, xv, pb, n, acc); break;
      default: gather_fma<T, GB, 8>(L, xv, pb, n, acc); break;
    }
  }
}

// Gather of one pattern group for the calling thread's staged point into ws[.][s][k]: the CSR row
// [p0, p1) staged in LDS in chunks of at most kGatherMax entries. Starts after a barrier that ends
// every earlier read of gcol / gval; ends without a barrier (the caller publishes ws).
template <typename T, int GB>
__device__ __attribute__((always_inline)) inline void gather_group(TileLds<T>& L, const c2_t<T>* __restrict__ xcol0,
                                                                   const int* __restrict__ col, const T* __restrict__ val,
                                                                   int p0, int p1, int K, size_t cstride, int s, int k,
                                                                   bool in) {
  GatherAcc<T> acc;
#pragma unroll
  for (int q = 0; q < kMaxGroup; ++q) acc.v[q] = cmk<T>(0, 0);
  for (int c0 = p0; c0 < p1; c0 += kGatherMax) {
    const int c1 = c0 + kGatherMax < p1 ? c0 + kGatherMax : p1;
    if (c0 > p0) __syncthreads();  // the previous chunk's reads are finished
    stage_csr<T>(L, col, val + (size_t)(c0 - p0) * K, c0, c1, K);
    __syncthreads();
    gather_point<T, GB>(L, xcol0, c1 - c0, K, cstride, acc);
  }
#pragma unroll
  for (int q = 0; q < kMaxGroup; ++q)
    if (q < K) L.ws[q][s][k] = in ? acc.v[q] : cmk<T>(0, 0);
}

// Result of one tile apply for the calling thread: S x and H x at (j, s, i).
// With a second term table (TWO) also hx2 = H x at the second table's fields (H0 part shared).
template <typename T> struct SH { c2_t<T> sx, hx, hx2; };

// Radial band taps of one (s, s') block at the calling thread's point: b[d] = B[s][s'][d][i].
template <typename T> struct Taps { T v[2 * kHB + 1]; };
template <typename T> struct CTaps { c2_t<T> v[2 * kHB + 1]; };

template <typename T>
__device__ inline void load_taps(Taps<T>& t, const T* p, int nr) {
#pragma unroll
  for (int d = 0; d < 2 * kHB + 1; ++d) t.v[d] = p[(size_t)d * nr];
}
template <typename T>
__device__ inline void load_ctaps(CTaps<T>& t, const c2_t<T>* p, int nr) {
#pragma unroll
  for (int d = 0; d < 2 * kHB + 1; ++d) t.v[d] = p[(size_t)d * nr];
}
// acc += sum_d t[d] * x[ii + d] (x: staged LDS row with the halo)
template <typename T>
__device__ inline c2_t<T> contract(const Taps<T>& t, const c2_t<T>* x, c2_t<T> acc) {
#pragma unroll
  for (int d = 0; d < 2 * kHB + 1; ++d) acc = rfma<T>(t.v[d], x[d], acc);
  return acc;
}
template <typename T>
__device__ inline c2_t<T> ccontract(const CTaps<T>& t, const c2_t<T>* x, c2_t<T> acc) {
#pragma unroll
  for (int d = 0; d < 2 * kHB + 1; ++d) acc = cfma<T>(t.v[d], x[d], acc);
  return acc;
}

// tl: the instance's term table in LDS (terms_to_lds). i0: first output point of the tile.
//
// Latency structure: every global load of a phase is issued before its first use, and the
// branches around loads depend only on the spinor component s (uniform over a wave: kStage threads
// per component) or on the tile's channel (uniform over the work-group), so they are scalar
// branches. A tile takes three dependent memory round trips when its channel's pattern row fits one
// gather batch: the staged value and the CSR row, the neighbour gather, then the taps (H0 / S taps
// issued before the barrier that publishes the staged values; coupling bands TR terms at a time).
// GB: gather batch; TR: coupling terms whose bands are loaded together (registers vs round trips).
template <typename T, bool TWO = false, int GB = kGatherBatch, int TR = 2>
__device__ inline SH<T> apply_tile(const DevOp<T>& op, const c2_t<T>* __restrict__ xinst, int j, int i0,
                                   const TermLds& tl, TileLds<T>& L, const TermLds* tl2 = nullptr) {
  constexpr int hb = kHB, nb = 2 * kHB + 1;
  const int nr = op.nr;
  const int s = __builtin_amdgcn_readfirstlane(threadIdx.x / kStage);
  const int k = threadIdx.x - s * kStage;
  const int i = i0 - hb + k;                            // staged point
  const bool in = i >= 0 && i < nr;                     // outside [0, nr) the staged values are 0
  const int ic = i < 0 ? 0 : (i >= nr ? nr - 1 : i);    // clamped point: loads stay in bounds
  const int kc = k < hb ? hb : (k >= kStage - hb ? kStage - hb - 1 : k);  // contraction window start + hb
  const size_t cstride = (size_t)2 * nr;
  const size_t bstride = (size_t)nb * nr;
  const c2_t<T>* xcol0 = xinst + (size_t)s * nr + ic;   // x[0][s][ic]; channel c at + c * cstride
  SH<T> out;
  out.sx = cmk<T>(0, 0);
  out.hx = cmk<T>(0, 0);
  out.hx2 = cmk<T>(0, 0);
  auto live_g = [&](int g) { return tl.g_live[g] != 0 || (TWO && tl2->g_live[g] != 0); };
  const c2_t<T> zero = cmk<T>(0, 0);

  // first pattern group: its CSR row staged with the channel's own value, its gather after one barrier
  const bool g0 = op.n_groups > 0 && live_g(0);
  int g0_p0 = 0, g0_p1 = 0, g0_K = 0;
  if (g0) {
    g0_K = tl.g_first[1];
    g0_p0 = op.g_rowptr[j];
    g0_p1 = op.g_rowptr[j + 1];
  }
  const T* g0_val = g0 ? op.g_val + op.g_voff[0] + (size_t)(g0_p0 - op.g_rowptr[0]) * g0_K : nullptr;
  c2_t<T> xown = xcol0[(size_t)j * cstride];
  if (!in) xown = zero;
  __syncthreads();  // the previous tile's LDS reads are finished
  L.xs[s][k] = xown;
  if (g0 && g0_p0 != g0_p1) gather_group<T, GB>(L, xcol0, op.g_col, g0_val, g0_p0, g0_p1, g0_K, cstride, s, k, in);

  // ---- H0 / S / channel taps of this kappa block: the real tap blocks this thread needs are listed
  // (uniform per wave; a complex channel block takes two, real and imaginary part), then loaded
  // kTapRound at a time with all loads of a round issued before any is used.
  constexpr int kTapSlots = 8, kTapRound = 2;
  const int kb = op.kblk_of[j];
  const T* sp[kTapSlots];
  // per slot: x component, destination (0 = H, 1 = H times i, 2 = S), element stride (1 real, 2 complex part)
  int sx2[kTapSlots], sdst[kTapSlots], sstr[kTapSlots];
  int ns = 0;
  auto add_slot = [&](const T* ptr, int s2, int dst, int str) {
#pragma unroll
    for (int q = 0; q < kTapSlots; ++q)
      if (q == ns) { sp[q] = ptr; sx2[q] = s2; sdst[q] = dst; sstr[q] = str; }
    ++ns;
  };
  // slot pointers are uniform (block starts); the thread's point is added at the load
#pragma unroll
  for (int s2 = 0; s2 < 2; ++s2) {
    const size_t blk = ((size_t)kb * 4 + s * 2 + s2) * bstride;
    if (op.n_h > 0 && (op.pq_h || s2 == s)) add_slot(op.h_blk + blk, s2, 0, 1);
    if (op.n_s > 0 && (op.pq_s || s2 == s)) add_slot(op.s_blk + blk, s2, 2, 1);
    if (op.has_chan && (op.pq_chan || s2 == s)) {
      const T* cp = reinterpret_cast<const T*>(op.h_chan + ((size_t)j * 4 + s * 2 + s2) * bstride);
      add_slot(cp, s2, 0, 2);
      add_slot(cp + 1, s2, 1, 2);
    }
  }
#pragma unroll
  for (int r = 0; r < kTapSlots / kTapRound; ++r) {
    Taps<T> tt[kTapRound];
#pragma unroll
    for (int q = 0; q < kTapRound; ++q) {
      const int sl = r * kTapRound + q;
      if (sl < ns) {
        const T* p = sp[sl] + (size_t)ic * sstr[sl];
        const size_t dstep = (size_t)nr * sstr[sl];
#pragma unroll
        for (int d = 0; d < nb; ++d) tt[q].v[d] = p[d * dstep];
      }
    }
    if (r == 0) __syncthreads();  // staged values visible (the first round's loads are already in flight)
#pragma unroll
    for (int q = 0; q < kTapRound; ++q) {
      const int sl = r * kTapRound + q;
      if (sl < ns) {
        const c2_t<T> a = contract<T>(tt[q], &L.xs[sx2[sl]][kc - hb], zero);
        if (sdst[sl] == 2) out.sx = cadd<T>(out.sx, a);
        else if (sdst[sl] == 1) out.hx = cadd<T>(out.hx, cmk<T>(-a.y, a.x));
        else out.hx = cadd<T>(out.hx, a);
      }
    }
  }
  if (op.n_s == 0) out.sx = L.xs[s][kc];
  if (TWO) out.hx2 = out.hx;

  // ---- coupling terms: stage the angular combinations of a pattern group, then the band
  // contractions, the bands of TR terms loaded together
  for (int gidx = 0; gidx < op.n_groups; ++gidx) {
    if (!live_g(gidx)) continue;  // uniform over the work-group
    const int f0 = tl.g_first[gidx], K = tl.g_first[gidx + 1] - f0;
    const int* rp = op.g_rowptr + (size_t)gidx * (op.nang + 1);
    const int p0 = rp[j], p1 = rp[j + 1];
    if (p0 == p1) continue;
    // the first group is staged together with the channel's own values above (one barrier less)
    if (gidx > 0) {
      const T* gv = op.g_val + op.g_voff[gidx] + (size_t)(p0 - rp[0]) * K;
      __syncthreads();
      gather_group<T, GB>(L, xcol0, op.g_col, gv, p0, p1, K, cstride, s, k, in);
      __syncthreads();
    }
#pragma unroll
    for (int q0 = 0; q0 < kMaxGroup; q0 += TR) {
      if (q0 < K) {
        Taps<T> tr[TR][2];
        int mask[TR], m[TR];
#pragma unroll
        for (int h = 0; h < TR; ++h) {
          const int q = q0 + h;
          m[h] = q < K ? tl.g_term[f0 + q] : 0;
          mask[h] = q < K ? (tl.g_mask[f0 + q] >> (2 * s)) & 3 : 0;
#pragma unroll
          for (int s2 = 0; s2 < 2; ++s2)
            if ((mask[h] >> s2) & 1)
              load_taps<T>(tr[h][s2], op.t_r + ((size_t)m[h] * 4 + s * 2 + s2) * bstride + ic, nr);
        }
#pragma unroll
        for (int h = 0; h < TR; ++h) {
          if (q0 + h < K) {
            c2_t<T> acc = zero;
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2)
              if ((mask[h] >> s2) & 1) acc = contract<T>(tr[h][s2], &L.ws[q0 + h][s2][kc - hb], acc);
            const double2 cf = tl.coef_f[m[h]];
            out.hx = cfma<T>(cmk<T>((T)cf.x, (T)cf.y), acc, out.hx);
            if (TWO) {
              const double2 cf2 = tl2->coef_f[m[h]];
              out.hx2 = cfma<T>(cmk<T>((T)cf2.x, (T)cf2.y), acc, out.hx2);
            }
          }
        }
      }
    }
  }
  return out;
}

// Element of x owned by the calling thread in the tile (j, it) of an instance; -1 for halo
// threads and points past nr.
__device__ inline long tile_elem(int nr, int j, int it) {
  const int s = threadIdx.x / kStage, k = threadIdx.x - s * kStage;
  const int i = it * kTileR - kHB + k;
  return (k >= kHB && k < kStage - kHB && i < nr) ? (long)j * 2 * nr + (long)s * nr + i : -1;
}

}  // namespace tdde
