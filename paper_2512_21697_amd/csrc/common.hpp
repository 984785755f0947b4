// Shared device-side definitions of the TDDE library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tdde {

constexpr int kThreads = 256;    // work-group size of every kernel
constexpr int kHB = 6;           // radial half-bandwidth: order-7 B-splines overlap 6 neighbours per side
constexpr int kMaxHB = kHB;
// A tile is one channel over kStage staged radial points per spinor component (2 x kStage = 256
// threads, one staged point each); its kTileR = kStage - 2 hb inner points are the outputs, the
// hb points on either side the halo of the radial band.
constexpr int kStage = kThreads / 2;
constexpr int kTileR = kStage - 2 * kHB;
constexpr int kMaxTerms = 128;   // largest number of coupling terms (the beyond-dipole operator: 24 per l)
constexpr int kMaxGroup = 8;     // coupling terms staged together (one group: union angular pattern)
constexpr int kMaxFields = 16;   // largest number of time functions per instance

template <typename T> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <typename T> using c2_t = typename cvec<T>::type;

template <typename T> __host__ __device__ inline c2_t<T> cmk(T re, T im) { c2_t<T> z; z.x = re; z.y = im; return z; }
template <typename T> __device__ inline c2_t<T> cadd(c2_t<T> a, c2_t<T> b) { return cmk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ inline c2_t<T> csub(c2_t<T> a, c2_t<T> b) { return cmk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ inline c2_t<T> cmul(c2_t<T> a, c2_t<T> b) {
  return cmk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// acc + a * b (complex a, complex b)
template <typename T> __device__ inline c2_t<T> cfma(c2_t<T> a, c2_t<T> b, c2_t<T> acc) {
  acc.x = fma(a.x, b.x, acc.x); acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y); acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
// acc - a * b (complex a, complex b)
template <typename T> __device__ inline c2_t<T> cfms(c2_t<T> a, c2_t<T> b, c2_t<T> acc) {
  acc.x = fma(-a.x, b.x, acc.x); acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(-a.x, b.y, acc.y); acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}
// acc + r * b (real r)
template <typename T> __device__ inline c2_t<T> rfma(T r, c2_t<T> b, c2_t<T> acc) {
  acc.x = fma(r, b.x, acc.x); acc.y = fma(r, b.y, acc.y);
  return acc;
}
template <typename T> __device__ inline c2_t<T> cscale(T r, c2_t<T> b) { return cmk<T>(r * b.x, r * b.y); }

// Loads and stores of device (global) memory through address-space-1 pointers. A pointer that
// reaches an outlined function is generic, and generic (flat) accesses share one wait counter with
// LDS accesses.
#define TDDE_GLOBAL __attribute__((address_space(1)))
typedef double gvd2 __attribute__((ext_vector_type(2)));
typedef float gvf2 __attribute__((ext_vector_type(2)));
__device__ __attribute__((always_inline)) inline double2 gld(const double2* p) {
  const gvd2 v = *(const TDDE_GLOBAL gvd2*)p;
  return make_double2(v.x, v.y);
}
__device__ __attribute__((always_inline)) inline float2 gld(const float2* p) {
  const gvf2 v = *(const TDDE_GLOBAL gvf2*)p;
  return make_float2(v.x, v.y);
}
__device__ __attribute__((always_inline)) inline void gst(double2* p, double2 x) {
  gvd2 v;
  v.x = x.x; v.y = x.y;
  *(TDDE_GLOBAL gvd2*)p = v;
}
__device__ __attribute__((always_inline)) inline void gst(float2* p, float2 x) {
  gvf2 v;
  v.x = x.x; v.y = x.y;
  *(TDDE_GLOBAL gvf2*)p = v;
}

// conj(a) * b accumulated in double
__device__ inline void dot_acc(double2& acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x); acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y); acc.y = fma(-a.y, b.x, acc.y);
}
__device__ inline void dot_acc(double2& acc, float2 a, float2 b) {
  dot_acc(acc, make_double2(a.x, a.y), make_double2(b.x, b.y));
}

// Device view of the operator (pointers into library-owned device memory).
template <typename T> struct DevOp {
  int nr, nang, hb, nb;        // nb = 2*hb + 1
  int n_h, n_s, has_chan;
  int pq_h, pq_s, pq_chan;     // 1 when the blocks couple s != s'
  int n_terms;
  int n_itiles;                // ceil(nr / kTileR) radial tiles per channel
  // H0 and S of every distinct kappa, the kappa polynomials summed on the host:
  // h_blk[kb][s][s'][d][i] = sum_n kappa^n h_n[s][s'][d][i] (likewise s_blk), kb = kblk_of[j]
  const int* kblk_of;          // [nang]
  const T* h_blk;              // [n_kblk][2][2][nb][nr] (null when n_h == 0)
  const c2_t<T>* h_chan;       // [nang][2][2][nb][nr]
  const T* s_blk;              // [n_kblk][2][2][nb][nr] (null when n_s == 0: S = I)
  // Terms grouped on the host (the union of their angular sparsity patterns) are staged together:
  // group g holds terms g_term[g_first[g] .. g_first[g+1]); its pattern is g_rowptr[g][nang+1]
  // (absolute offsets into g_col); the value of term k of the group at pattern entry p is
  // g_val[g_voff[g] + (p - g_rowptr[g][0]) * K + k], K = group size, with the kappa exponents
  // folded in: kappa_j^a * A[j][j'] * kappa_j'^b.
  int n_groups;
  const int* g_first;          // [n_groups + 1]
  const int* g_term;           // [n_terms]
  const int* g_rowptr;         // [n_groups][nang+1]
  const int* g_col;
  const long* g_voff;          // [n_groups]
  const T* g_val;
  const T* t_r;                // [n_terms][2][2][nb][nr]
  const int* t_mask;           // [n_terms] bit (2 s + s') set when block (s, s') of R_m is nonzero
  const int* t_field;          // [n_terms]
  const double2* t_coef;       // [n_terms] (double even for the FP32 copy)
};

// Tile t of one instance -> (channel j, radial tile it). The work-group that takes tile t is
// t mod G (G a multiple of 8, or the tile index itself in the standalone apply) and work-groups are
// dispatched round-robin over the 8 XCDs, so tile t runs on XCD t % 8. The first 8 floor(nit / 8)
// radial tiles are dealt in groups of 8 with the radial tile fastest: radial tile it of every
// channel runs on XCD it % 8, channel after channel, so the x tiles that the angular coupling of
// neighbouring channels reads again are in that XCD's L2. The remaining radial tiles follow,
// channel-major.
__device__ inline void tile_coords(int nang, int nit, int t, int& j, int& it) {
  const int n8 = nit & ~7;
  const int full = n8 * nang;
  if (t < full) {
    const int q = t / (8 * nang), r = t - q * 8 * nang;
    j = r >> 3;
    it = q * 8 + (r & 7);
  } else {
    const int rem = t - full, nl = nit - n8;
    j = rem / nl;
    it = n8 + (rem - j * nl);
  }
}

// Sum over the work-group of a complex (two doubles), fixed order: wave shuffles, then waves in
// order. lds holds 2 * kThreads / 64 doubles.
__device__ inline double2 wg_sum2(double2 v, double* lds) {
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) { lds[2 * wid] = v.x; lds[2 * wid + 1] = v.y; }
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
  for (int k = 0; k < kThreads / 64; ++k) { s.x += lds[2 * k]; s.y += lds[2 * k + 1]; }
  __syncthreads();
  return s;
}

// Grid-wide barrier for a co-resident (cooperatively launched) grid.
//
// Arrivals are spread over kBarGroups counters (work-group g arrives on counter g % kBarGroups),
// each in its own 256-byte line, so no more than nwg / kBarGroups atomics queue on one address;
// the last arrival of a group arrives on the top counter, and the last of those publishes the new
// generation into one flag line per group, which that group's work-groups poll. Counters are reset
// by their last arrival before the generation is published, so the next barrier finds them at zero.
// Ordering: arrival is a release (the work-group's writes become visible device-wide, across
// XCDs); the group and top finishers acquire before passing on; pollers use relaxed loads (an
// acquire per poll would invalidate the XCD's L2 under the working work-groups) and one acquire
// fence once the generation has changed. The spin is bounded: on time-out the error word is set
// and every later barrier returns false at once, so the kernel always terminates.
constexpr int kBarGroups = 16;
constexpr int kBarLine = 64;  // words per 256-byte line
constexpr int kBarTop = kBarGroups * kBarLine;
constexpr int kBarFlag0 = (kBarGroups + 1) * kBarLine;
constexpr int kBarErr = (2 * kBarGroups + 1) * kBarLine;
constexpr int kBarWords = (2 * kBarGroups + 2) * kBarLine;  // zeroed before every launch
constexpr unsigned kSpinLimit = 1u << 24;

struct GridBar {
  unsigned* w;     // kBarWords words
  unsigned nwg;    // work-groups in the grid
  unsigned gen;    // generations passed (all threads keep the same count)
  bool failed;
};

// watch: optional device counter read by thread 0 after the barrier (every work-group's updates
// before the barrier are visible); its value is returned in *watch_val for the whole work-group.
__device__ inline bool grid_barrier(GridBar& gb, const int* watch = nullptr, int* watch_val = nullptr) {
  __shared__ unsigned bar_ok;
  __shared__ int watch_s;
  if (gb.failed) return false;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned* w = gb.w;
    const unsigned K = gb.nwg < (unsigned)kBarGroups ? gb.nwg : (unsigned)kBarGroups;
    const unsigned g = blockIdx.x % K;
    const unsigned members = (gb.nwg - g + K - 1) / K;
    const unsigned target = gb.gen + 1;
    unsigned ok = 1;
    const unsigned a = __hip_atomic_fetch_add(&w[g * kBarLine], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    bool publish = false;
    if (a == members - 1) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(&w[g * kBarLine], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned t = __hip_atomic_fetch_add(&w[kBarTop], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      if (t == K - 1) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __hip_atomic_store(&w[kBarTop], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        for (unsigned k = 0; k < K; ++k)
          __hip_atomic_store(&w[kBarFlag0 + k * kBarLine], target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        publish = true;
      }
    }
    if (!publish) {
      unsigned spins = 0;
      while (__hip_atomic_load(&w[kBarFlag0 + g * kBarLine], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != target) {
        __builtin_amdgcn_s_sleep(1);
        ++spins;
        if ((spins & 255u) == 0 &&
            (spins > kSpinLimit || __hip_atomic_load(&w[kBarErr], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)) {
          __hip_atomic_store(&w[kBarErr], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // see every arrival's writes (all XCDs)
    }
    bar_ok = ok;
    if (watch != nullptr) watch_s = __hip_atomic_load(watch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  gb.gen++;
  if (bar_ok == 0u) gb.failed = true;
  if (watch_val != nullptr) *watch_val = watch_s;
  return !gb.failed;
}

// Midpoint time of step `step` on the axis t = t0 + step * dt (Sec. 2.4 midpoint rule), formed with an
// explicit multiply-add so every kernel that evaluates it gets the same bits.
__device__ inline double mid_time(double t0, int step, double dt) { return fma((double)step, dt, t0) + 0.5 * dt; }

// Time function of eq. ndpPot (dipole limit): amp * env * sin(omega t + phase) on (0, T).
struct PulseDev { double amp, T, omega, phase; int envelope, pad; };
__device__ inline double pulse_eval(const PulseDev& p, double t) {
  if (!(t > 0.0 && t < p.T)) return 0.0;
  double env = 1.0;
  if (p.envelope) { double s = sin(M_PI * t / p.T); env = s * s; }
  return p.amp * env * sin(p.omega * t + p.phase);
}

}  // namespace tdde
