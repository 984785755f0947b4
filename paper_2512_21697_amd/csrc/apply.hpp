// Matrix-free apply of S and H(t) on one (instance, channel, radial tile) of x[b][j][s][i].
//
// eq. fullH: (H x)[j][s][i] = sum_{s',d} H0_j[s][s'][d][i] x[j][s'][i+d]
//                           + sum_m coef_m f_m sum_{j'} (K^a A_m K^b)[j][j'] sum_{s',d} R_m[s][s'][d][i] x[j'][s'][i+d]
// with H0_j = sum_n kappa_j^n h_n (+ per-channel complex band), S_j = sum_n kappa_j^n s_n or I; the
// kappa polynomials are summed once per distinct kappa on the host, so a tap is one band load.
//
// Work-group layout: 256 threads = 2 components x 128 radial points; thread (s, ii) owns
// y[j][s][i0 + ii]. The x tile of channel j (with a halo of hb points) is staged in LDS; the
// angular combinations w_m = sum_j' A_m[j][j'] x[j'] of all terms of one group (terms sharing the
// union of their sparsity patterns) are staged in LDS together (each neighbouring x value is read
// once per group), so the radial band contraction reads LDS and the angular gather is not repeated
// per radial tap or per term.
#pragma once
#include "common.hpp"

namespace tdde {

constexpr int kGatherMax = 64;  // CSR entries of one pattern row staged in LDS at a time

template <typename T> struct TileLds {
  c2_t<T> xs[2][kHalo];
  c2_t<T> ws[kMaxGroup][2][kHalo];
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

// CSR row [p0, p1) of one pattern group (column indices and the K term values of every entry)
// into LDS; at most kGatherMax entries (rows with more take the direct path of stage_gather).
template <typename T>
__device__ inline void stage_csr(TileLds<T>& L, const int* __restrict__ col, const T* __restrict__ val, int p0, int p1,
                                 int K) {
  const int n = p1 - p0;
  if (n > kGatherMax) return;
  for (int k = threadIdx.x; k < n; k += kThreads) L.gcol[k] = col[p0 + k];
  for (int k = threadIdx.x; k < n * K; k += kThreads) L.gval[k] = val[k];
}

// Stage w_k[s'][.] = sum_p val[p * K + k] * x[col[p]][s'][.] for the K terms of one pattern group and
// the CSR row [p0, p1): every neighbouring x value is loaded once for all K terms. The CSR row is
// read from LDS (stage_csr, after a barrier) when it fits, else from global memory; the neighbour
// loads of GB entries are issued together before they are used (GB trades registers for fewer
// dependent memory round trips).
template <typename T, int GB>
__device__ inline void stage_gather(TileLds<T>& L, const c2_t<T>* __restrict__ xinst, const int* __restrict__ col,
                                    const T* __restrict__ val, int p0, int p1, int K, int i0, int nr) {
  constexpr int hb = kHB;
  constexpr int w = kTileR + 2 * hb;
  const size_t cstride = (size_t)2 * nr;
  const int n = p1 - p0;
  const bool in_lds = n <= kGatherMax;
  for (int k = threadIdx.x; k < 2 * w; k += kThreads) {
    const int s = k / w, kk = k - s * w, gi = i0 - hb + kk;
    const bool in = gi >= 0 && gi < nr;
    const int gic = in ? gi : 0;
    c2_t<T> acc[kMaxGroup];
#pragma unroll
    for (int q = 0; q < kMaxGroup; ++q) acc[q] = cmk<T>(0, 0);
    for (int pb = 0; pb < n; pb += GB) {
      c2_t<T> xv[GB];
#pragma unroll
      for (int u = 0; u < GB; ++u) {
        const int p = pb + u < n ? pb + u : n - 1;
        const int c = in_lds ? L.gcol[p] : col[p0 + p];
        xv[u] = xinst[(size_t)c * cstride + (size_t)s * nr + gic];
      }
#pragma unroll
      for (int u = 0; u < GB; ++u) {
        if (pb + u < n) {
          const T* v = (in_lds ? L.gval : val) + (size_t)(pb + u) * K;
#pragma unroll
          for (int q = 0; q < kMaxGroup; ++q)
            if (q < K) acc[q] = rfma<T>(v[q], xv[u], acc[q]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kMaxGroup; ++q)
      if (q < K) L.ws[q][s][kk] = in ? acc[q] : cmk<T>(0, 0);
  }
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

// tl: the instance's term table in LDS (terms_to_lds).
//
// Latency structure: every global load of a phase is issued before its first use, and the
// branches around loads depend only on the spinor component s, which is uniform over a wave
// (128 threads per component), so they are scalar branches: H0/S taps are loaded before the
// staging barrier is passed, coupling bands TR terms at a time.
// GB: gather batch; TR: coupling terms whose bands are loaded together (registers vs round trips).
template <typename T, bool TWO = false, int GB = 4, int TR = 2>
__device__ inline SH<T> apply_tile(const DevOp<T>& op, const c2_t<T>* __restrict__ xinst, int j, int i0,
                                   const TermLds& tl, TileLds<T>& L, const TermLds* tl2 = nullptr) {
  constexpr int hb = kHB, nb = 2 * kHB + 1;
  const int nr = op.nr;
  const int s = __builtin_amdgcn_readfirstlane(threadIdx.x / kTileR);
  const int ii = threadIdx.x - s * kTileR, i = i0 + ii;
  const bool live = i < nr;
  const int ic = live ? i : nr - 1;  // clamped point: loads stay in bounds, results unused
  const size_t cstride = (size_t)2 * nr;
  const size_t bstride = (size_t)nb * nr;
  SH<T> out;
  out.sx = cmk<T>(0, 0);
  out.hx = cmk<T>(0, 0);
  out.hx2 = cmk<T>(0, 0);
  auto live_g = [&](int g) { return tl.g_live[g] != 0 || (TWO && tl2->g_live[g] != 0); };

  // first pattern group: its CSR row staged with the channel tile, its gather after one barrier
  const bool g0 = op.n_groups > 0 && live_g(0);
  int g0_p0 = 0, g0_p1 = 0, g0_K = 0;
  if (g0) {
    g0_K = tl.g_first[1];
    g0_p0 = op.g_rowptr[j];
    g0_p1 = op.g_rowptr[j + 1];
  }
  const T* g0_val = g0 ? op.g_val + op.g_voff[0] + (size_t)(g0_p0 - op.g_rowptr[0]) * g0_K : nullptr;
  __syncthreads();
  stage_channel<T>(L.xs, xinst + (size_t)j * cstride, i0, nr);
  if (g0 && g0_p0 != g0_p1) {
    stage_csr<T>(L, op.g_col, g0_val, g0_p0, g0_p1, g0_K);
    __syncthreads();
    stage_gather<T, GB>(L, xinst, op.g_col, g0_val, g0_p0, g0_p1, g0_K, i0, nr);
  }

  // ---- H0 / S / channel taps of this kappa block: the real tap blocks this thread needs are listed
  // (uniform per wave; a complex channel block takes two, real and imaginary part), then loaded
  // kTapRound at a time with all loads of a round issued before any is used.
  constexpr int kTapSlots = 8, kTapRound = 4;
  const int kb = op.kblk_of[j];
  const T* sp[kTapSlots];
  // per slot: x component, destination (0 = H, 1 = H times i, 2 = S), element stride (1 real, 2 complex part)
  int sx2[kTapSlots], sdst[kTapSlots], sstr[kTapSlots];
  int ns = 0;
  auto add_slot = [&](const T* ptr, int s2, int dst, int str) {
#pragma unroll
    for (int k = 0; k < kTapSlots; ++k)
      if (k == ns) { sp[k] = ptr; sx2[k] = s2; sdst[k] = dst; sstr[k] = str; }
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
    for (int k = 0; k < kTapRound; ++k) {
      const int sl = r * kTapRound + k;
      if (sl < ns) {
        const T* p = sp[sl] + (size_t)ic * sstr[sl];
        const size_t dstep = (size_t)nr * sstr[sl];
#pragma unroll
        for (int d = 0; d < nb; ++d) tt[k].v[d] = p[d * dstep];
      }
    }
    if (r == 0) __syncthreads();  // staged x visible (the first round's loads are already in flight)
#pragma unroll
    for (int k = 0; k < kTapRound; ++k) {
      const int sl = r * kTapRound + k;
      if (sl < ns) {
        const c2_t<T> a = contract<T>(tt[k], &L.xs[sx2[sl]][ii], cmk<T>(0, 0));
        if (sdst[sl] == 2) out.sx = cadd<T>(out.sx, a);
        else if (sdst[sl] == 1) out.hx = cadd<T>(out.hx, cmk<T>(-a.y, a.x));
        else out.hx = cadd<T>(out.hx, a);
      }
    }
  }
  if (op.n_s == 0) out.sx = L.xs[s][ii + hb];
  if (TWO) out.hx2 = out.hx;

  // ---- coupling terms: stage the angular combinations of a pattern group, then the band
  // contractions, the bands of TR terms loaded together
  for (int gidx = 0; gidx < op.n_groups; ++gidx) {
    if (!live_g(gidx)) continue;  // uniform over the work-group
    const int f0 = tl.g_first[gidx], K = tl.g_first[gidx + 1] - f0;
    const int* rp = op.g_rowptr + (size_t)gidx * (op.nang + 1);
    const int p0 = rp[j], p1 = rp[j + 1];
    if (p0 == p1) continue;
    // the first group is staged together with the channel tile above (one barrier less)
    if (gidx > 0) {
      const T* gv = op.g_val + op.g_voff[gidx] + (size_t)(p0 - rp[0]) * K;
      __syncthreads();
      stage_csr<T>(L, op.g_col, gv, p0, p1, K);
      __syncthreads();
      stage_gather<T, GB>(L, xinst, op.g_col, gv, p0, p1, K, i0, nr);
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
            c2_t<T> acc = cmk<T>(0, 0);
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2)
              if ((mask[h] >> s2) & 1) acc = contract<T>(tr[h][s2], &L.ws[q0 + h][s2][ii], acc);
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

}  // namespace tdde
