// Matrix-free apply of S and H(t) on one (instance, channel, radial tile) of x[b][j][s][i].
//
// eq. fullH: (H x)[j][s][i] = sum_{s',d} H0_j[s][s'][d][i] x[j][s'][i+d]
//                           + sum_m coef_m f_m sum_{j'} (K^a A_m K^b)[j][j'] sum_{s',d} R_m[s][s'][d][i] x[j'][s'][i+d]
// with H0_j = sum_n kappa_j^n h_n (+ per-channel complex band), S_j = sum_n kappa_j^n s_n or I.
//
// Work-group layout: 256 threads = 2 components x 128 radial points; thread (s, ii) owns
// y[j][s][i0 + ii]. The x tile of channel j (with a halo of hb points) is staged in LDS; the
// angular combinations w_m = sum_j' A_m[j][j'] x[j'] of all terms sharing one sparsity pattern are
// staged in LDS together (each neighbouring x value is read once per pattern), so the radial band
// contraction reads LDS and the angular gather is not repeated per radial tap or per term.
#pragma once
#include "common.hpp"

namespace tdde {

template <typename T> struct TileLds {
  c2_t<T> xs[2][kHalo];
  c2_t<T> ws[kMaxGroup][2][kHalo];
};

// Stage v[s'][i0-hb .. i0+kTileR+hb) of one channel into dst (zero outside [0, nr)).
template <typename T>
__device__ inline void stage_channel(c2_t<T> (*dst)[kHalo], const c2_t<T>* __restrict__ chan, int i0, int nr) {
  constexpr int hb = kHB;
  constexpr int w = kTileR + 2 * hb;
  for (int k = threadIdx.x; k < 2 * w; k += kThreads) {
    const int s = k / w, kk = k - s * w, gi = i0 - hb + kk;
    c2_t<T> v = cmk<T>(0, 0);
    if (gi >= 0 && gi < nr) v = chan[(size_t)s * nr + gi];
    dst[s][kk] = v;
  }
}

// Stage w_k[s'][.] = sum_p val[p * K + k] * x[col[p]][s'][.] for the K terms of one pattern group and
// the CSR row [p0, p1): every neighbouring x value is loaded once for all K terms.
template <typename T>
__device__ inline void stage_gather(c2_t<T> (*dst)[2][kHalo], const c2_t<T>* __restrict__ xinst, const int* __restrict__ col,
                                    const T* __restrict__ val, int p0, int p1, int K, int i0, int nr) {
  constexpr int hb = kHB;
  constexpr int w = kTileR + 2 * hb;
  const size_t cstride = (size_t)2 * nr;
  for (int k = threadIdx.x; k < 2 * w; k += kThreads) {
    const int s = k / w, kk = k - s * w, gi = i0 - hb + kk;
    c2_t<T> acc[kMaxGroup];
#pragma unroll
    for (int q = 0; q < kMaxGroup; ++q) acc[q] = cmk<T>(0, 0);
    if (gi >= 0 && gi < nr) {
#pragma unroll 4
      for (int p = p0; p < p1; ++p) {
        const c2_t<T> xv = xinst[(size_t)col[p] * cstride + (size_t)s * nr + gi];
        const T* v = val + (size_t)(p - p0) * K;
#pragma unroll
        for (int q = 0; q < kMaxGroup; ++q)
          if (q < K) acc[q] = rfma<T>(v[q], xv, acc[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < kMaxGroup; ++q)
      if (q < K) dst[q][s][kk] = acc[q];
  }
}

// Result of one tile apply for the calling thread: S x and H x at (j, s, i).
template <typename T> struct SH { c2_t<T> sx, hx; };

// coef_f: LDS array [n_terms] of coef_m * f_{field_m}(t) for this instance.
template <typename T>
__device__ inline SH<T> apply_tile(const DevOp<T>& op, const c2_t<T>* __restrict__ xinst, int j, int i0,
                                   const double2* coef_f, TileLds<T>& L) {
  constexpr int hb = kHB, nb = 2 * kHB + 1;
  const int nr = op.nr;
  const int s = threadIdx.x / kTileR, ii = threadIdx.x - s * kTileR, i = i0 + ii;
  const bool live = i < nr;
  const size_t cstride = (size_t)2 * nr;
  SH<T> out;
  out.sx = cmk<T>(0, 0);
  out.hx = cmk<T>(0, 0);

  __syncthreads();
  stage_channel<T>(L.xs, xinst + (size_t)j * cstride, i0, nr);
  if (op.n_groups > 0) {
    const int K0 = op.g_first[1];
    const int p0 = op.g_rowptr[j], p1 = op.g_rowptr[j + 1];
    bool any = false;
    for (int q = 0; q < K0; ++q) {
      const double2 cf = coef_f[op.g_term[q]];
      any = any || cf.x != 0.0 || cf.y != 0.0;
    }
    if (p0 != p1 && any)
      stage_gather<T>(L.ws, xinst, op.g_col, op.g_val + op.g_voff[0] + (size_t)(p0 - op.g_rowptr[0]) * K0, p0, p1, K0,
                      i0, nr);
  }
  __syncthreads();

  const T kap = op.kappa[j];
  if (live) {
    const size_t bstride = (size_t)nb * nr;
    // H0 (kappa polynomial, Horner) and S; taps fully unrolled, polynomial coefficients loaded
    // before the Horner chain so all loads of a tap are in flight together
    const int n_h = op.n_h, n_s = op.n_s;
    for (int s2 = 0; s2 < 2; ++s2) {
      const bool do_h = n_h > 0 && (op.pq_h || s2 == s);
      const bool do_c = op.has_chan && (op.pq_chan || s2 == s);
      const bool do_s = n_s > 0 && (op.pq_s || s2 == s);
      if (!(do_h || do_c || do_s)) continue;
      const size_t blk = (size_t)(s * 2 + s2) * bstride + i;
      const T* hp = op.h_poly + blk;
      const T* sp = op.s_poly + blk;
      const c2_t<T>* hc = op.h_chan + (size_t)j * 4 * bstride + blk;
#pragma unroll
      for (int d = -hb; d <= hb; ++d) {
        const c2_t<T> xv = L.xs[s2][ii + hb + d];
        const size_t off = (size_t)(d + hb) * nr;
        if (do_h) {
          T cf[4];
#pragma unroll
          for (int n = 0; n < 4; ++n) cf[n] = n < n_h ? hp[(size_t)n * 4 * bstride + off] : (T)0;
          const T tap = fma(fma(fma(cf[3], kap, cf[2]), kap, cf[1]), kap, cf[0]);
          out.hx = rfma<T>(tap, xv, out.hx);
        }
        if (do_c) out.hx = cfma<T>(hc[off], xv, out.hx);
        if (do_s) {
          T cf[3];
#pragma unroll
          for (int n = 0; n < 3; ++n) cf[n] = n < n_s ? sp[(size_t)n * 4 * bstride + off] : (T)0;
          const T tap = fma(fma(cf[2], kap, cf[1]), kap, cf[0]);
          out.sx = rfma<T>(tap, xv, out.sx);
        }
      }
    }
    if (op.n_s == 0) out.sx = L.xs[s][ii + hb];
  }

  // coupling terms: stage the angular combinations of a pattern group, then the band contractions
  for (int gidx = 0; gidx < op.n_groups; ++gidx) {
    const int f0 = op.g_first[gidx], K = op.g_first[gidx + 1] - f0;
    const int* rp = op.g_rowptr + (size_t)gidx * (op.nang + 1);
    const int p0 = rp[j], p1 = rp[j + 1];
    bool any = false;
    for (int q = 0; q < K; ++q) {
      const double2 cf = coef_f[op.g_term[f0 + q]];
      any = any || cf.x != 0.0 || cf.y != 0.0;
    }
    if (p0 == p1 || !any) continue;  // uniform over the work-group
    // the first group is staged together with the channel tile above (one barrier less)
    if (gidx > 0) {
      __syncthreads();
      stage_gather<T>(L.ws, xinst, op.g_col, op.g_val + op.g_voff[gidx] + (size_t)(p0 - rp[0]) * K, p0, p1, K, i0, nr);
      __syncthreads();
    }
    if (live) {
      const size_t bstride = (size_t)nb * nr;
      for (int q = 0; q < K; ++q) {
        const int m = op.g_term[f0 + q];
        const double2 cf = coef_f[m];
        if (cf.x == 0.0 && cf.y == 0.0) continue;
        const T* R = op.t_r + (size_t)m * 4 * bstride;
        const bool pq = op.t_pq[m] != 0;
        c2_t<T> acc = cmk<T>(0, 0);
        for (int s2 = 0; s2 < 2; ++s2) {
          if (!pq && s2 != s) continue;
          const T* Rb = R + (size_t)(s * 2 + s2) * bstride + i;
#pragma unroll
          for (int d = -hb; d <= hb; ++d) acc = rfma<T>(Rb[(size_t)(d + hb) * nr], L.ws[q][s2][ii + hb + d], acc);
        }
        out.hx = cfma<T>(cmk<T>((T)cf.x, (T)cf.y), acc, out.hx);
      }
    }
  }
  return out;
}

}  // namespace tdde
