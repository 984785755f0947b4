// Shared device-side definitions of the TDDE library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tdde {

constexpr int kThreads = 256;    // work-group size of every kernel
constexpr int kTileR = 128;      // radial points per tile (x 2 spinor components = 256 threads)
constexpr int kHB = 6;           // radial half-bandwidth: order-7 B-splines overlap 6 neighbours per side
constexpr int kMaxHB = kHB;
constexpr int kMaxTerms = 32;    // largest number of coupling terms
constexpr int kMaxGroup = 8;     // coupling terms staged together (same angular sparsity pattern)
constexpr int kMaxFields = 16;   // largest number of time functions per instance
constexpr int kHalo = kTileR + 2 * kMaxHB;

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
// acc + r * b (real r)
template <typename T> __device__ inline c2_t<T> rfma(T r, c2_t<T> b, c2_t<T> acc) {
  acc.x = fma(r, b.x, acc.x); acc.y = fma(r, b.y, acc.y);
  return acc;
}
template <typename T> __device__ inline c2_t<T> cscale(T r, c2_t<T> b) { return cmk<T>(r * b.x, r * b.y); }

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
  int n_itiles;                // ceil(nr / kTileR)
  const T* kappa;              // [nang]
  const T* h_poly;             // [n_h][2][2][nb][nr]
  const c2_t<T>* h_chan;       // [nang][2][2][nb][nr]
  const T* s_poly;             // [n_s][2][2][nb][nr]
  // Terms with one angular sparsity pattern form a group and are staged together:
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
  const int* t_pq;             // [n_terms]
  const int* t_field;          // [n_terms]
  const double2* t_coef;       // [n_terms] (double even for the FP32 copy)
};

// Sum of a double over the work-group (fixed order: wave shuffles, then waves in order).
__device__ inline double wg_sum(double v, double* lds) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < kThreads / 64; ++k) s += lds[k];
  __syncthreads();
  return s;
}

__device__ inline double2 wg_sum2(double2 v, double* lds) {
  return make_double2(wg_sum(v.x, lds), wg_sum(v.y, lds));
}

// Grid-wide barrier for a co-resident (cooperatively launched) grid.
// bar[0] = arrival count, bar[1] = generation, bar[2] = error flag. Arrival is a release (the
// work-group's writes become visible device-wide, across XCDs); waiting polls with relaxed loads
// (an acquire per poll would invalidate the XCD's L2 under the working work-groups) and issues one
// acquire fence after the generation changes. The spin is bounded: on time-out the error flag is
// raised and every later barrier returns at once, so the kernel always terminates.
constexpr unsigned kSpinLimit = 1u << 24;
__device__ inline bool grid_barrier(unsigned* bar, unsigned nwg) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nwg - 1) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned spins = 0;
      while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit ||
            __hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
          __hip_atomic_store(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // see every arrival's writes (all XCDs)
  }
  __syncthreads();
  return __hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
}

// Time function of eq. ndpPot (dipole limit): amp * env * sin(omega t + phase) on (0, T).
struct PulseDev { double amp, T, omega, phase; int envelope, pad; };
__device__ inline double pulse_eval(const PulseDev& p, double t) {
  if (!(t > 0.0 && t < p.T)) return 0.0;
  double env = 1.0;
  if (p.envelope) { double s = sin(M_PI * t / p.T); env = s * s; }
  return p.amp * env * sin(p.omega * t + p.phase);
}

}  // namespace tdde
