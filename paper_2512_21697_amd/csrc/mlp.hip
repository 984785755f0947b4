// Learned initial guess (include/tdde_mlp.h): fused BF16-MFMA forward, backward GEMMs, Adam.
//
// MFMA v_mfma_f32_16x16x32_bf16 operand layout (wave64, lane l, n = l % 16, g = l / 16):
//   A[m = n][k = 8 g + j], B[k = 8 g + j][n], j = 0..7;  D[m = 4 g + i][n], i = 0..3.
// The forward pass keeps data rows on n and hidden units on the MFMA m dimension (it computes
// Z^T = W X^T), so every layer's output lands in the layout the next layer consumes:
// lane (g, n) holds, for data row n, hidden units 16 t + 4 g + i of output tile t. Layer 2's
// K index is permuted so that its B operand for K-step kk is exactly the layer-1 outputs of
// tiles 2kk and 2kk+1 already held by the lane; W2 is stored in LDS in the same permuted order
// (see refresh_kernel), so no activation moves between lanes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tdde_mlp.h"
#include "common.hpp"

using tdde::PulseDev;
using tdde::pulse_eval;

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int H = 256, F = 32;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + H * F, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H, OFF_W3 = OFF_B2 + H,
              OFF_B3 = OFF_W3 + 2 * H, N_PARAM = OFF_B3 + 2;
constexpr int N_SKIP = 17;     // c[2][4][2] (re, im) and sigma, FP64
constexpr int RAW = 16;        // doubles per raw training sample
constexpr int W2P_VEC = 16 * 8 * 64;  // bf16x8 entries of the permuted W2

struct Weights {
  const bf16* W1;       // [H][F]
  const bf16x8* W2p;    // permuted, W2P_VEC entries
  const float* P;       // FP32 master (biases)
  const float* W3r;     // [2][H] W3 rounded to bf16, as float
  const double* skip;   // c[2][4][2], sigma
};

__device__ inline float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ inline float dsilu(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}
__device__ inline float bfr(float x) { return (float)(bf16)x; }

struct FwdArgs {
  long M;
  double tau;
  // RAW source (training)
  const double* raw;
  // history source (inference)
  const double2* hist0;
  const double2* hist1;
  const double2* hist2;
  const double2* hist3;
  long E;
  int nr, n_fields;
  const PulseDev* pulses;
  double t_n, dt;
  double2* guess;
  // outputs
  float* out;   // [M][2] prediction of psi_{n+1} / rho (training)
  // training stash
  float* Z1; float* Z2;      // [M][H]
  bf16* H1; bf16* H2;        // [M][H]
  bf16* X;                   // [M][F]
  float* U;                  // [M][8] skip inputs
  float* T;                  // [M][2] targets
  int* S;                    // [M]
};

// Features of one row for the calling lane: x[8 g .. 8 g + 7] plus the skip data (g == 0 lanes).
template <bool FROM_RAW>
__device__ inline bf16x8 row_features(const FwdArgs& a, long r, int g, bool valid, double2 (&psi)[4], double& rho,
                                      int& s, double2& tgt) {
  bf16x8 x;
#pragma unroll
  for (int j = 0; j < 8; ++j) x[j] = (bf16)0.0f;
  rho = 1.0;
  s = 0;
  tgt = make_double2(0, 0);
  if (!valid) return x;
  double fh = 0.0, fm = 0.0;
  if (FROM_RAW) {
    const double* p = a.raw + r * RAW;
#pragma unroll
    for (int k = 0; k < 4; ++k) psi[k] = make_double2(p[2 * k], p[2 * k + 1]);
    tgt = make_double2(p[8], p[9]);
    fh = p[10];
    fm = p[11];
    s = p[12] != 0.0 ? 1 : 0;
  } else {
    psi[0] = a.hist0[r];
    psi[1] = a.hist1[r];
    psi[2] = a.hist2[r];
    psi[3] = a.hist3[r];
    const long b = r / a.E, e = r - b * a.E;
    s = (int)((e / a.nr) & 1);
    const PulseDev pu = a.pulses[b * a.n_fields];
    fh = pulse_eval(pu, a.t_n + 0.5 * a.dt);
    fm = pulse_eval(pu, a.t_n - 0.5 * a.dt);
  }
  rho = sqrt(psi[0].x * psi[0].x + psi[0].y * psi[0].y + psi[1].x * psi[1].x + psi[1].y * psi[1].y + a.tau * a.tau);
  const double ir = 1.0 / rho;
  if (g == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      x[2 * k] = (bf16)(float)(psi[k].x * ir);
      x[2 * k + 1] = (bf16)(float)(psi[k].y * ir);
    }
  } else if (g == 1) {
    x[0] = (bf16)(float)fh;
    x[1] = (bf16)(float)fm;
    x[2] = (bf16)(float)s;
  }
  return x;
}

template <bool TRAIN>
__global__ __launch_bounds__(256) void mlp_fwd_kernel(Weights w, FwdArgs a) {
  __shared__ bf16x8 W2s[W2P_VEC];  // 128 KiB
  __shared__ float W3s[2 * H], b1s[H], b2s[H];
  for (int i = threadIdx.x; i < W2P_VEC; i += blockDim.x) W2s[i] = w.W2p[i];
  for (int i = threadIdx.x; i < 2 * H; i += blockDim.x) W3s[i] = w.W3r[i];
  for (int i = threadIdx.x; i < H; i += blockDim.x) {
    b1s[i] = w.P[OFF_B1 + i];
    b2s[i] = w.P[OFF_B2 + i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, n = lane & 15;
  // layer-1 A operands: W1[16 t + n][8 g + j]
  bf16x8 w1f[16];
#pragma unroll
  for (int t = 0; t < 16; ++t)
#pragma unroll
    for (int j = 0; j < 8; ++j) w1f[t][j] = w.W1[(16 * t + n) * F + 8 * g + j];
  const float b30 = w.P[OFF_B3], b31 = w.P[OFF_B3 + 1];
  const long npass = (a.M + 31) / 32;
  for (long pass = (long)blockIdx.x * 4 + wave; pass < npass; pass += (long)gridDim.x * 4) {
    const long row0 = pass * 32;
    bf16x8 xb[2];
    double2 psi[2][4];
    double rho[2];
    int sflag[2];
    double2 tgt[2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const long r = row0 + 16 * rt + n;
      if (TRAIN)
        xb[rt] = row_features<true>(a, r, g, r < a.M, psi[rt], rho[rt], sflag[rt], tgt[rt]);
      else
        xb[rt] = row_features<false>(a, r, g, r < a.M, psi[rt], rho[rt], sflag[rt], tgt[rt]);
      if (TRAIN && r < a.M) {
        *reinterpret_cast<bf16x8*>(a.X + r * F + 8 * g) = xb[rt];
        if (g == 0) {
          const double ir = 1.0 / rho[rt];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            a.U[r * 8 + 2 * k] = (float)(psi[rt][k].x * ir);
            a.U[r * 8 + 2 * k + 1] = (float)(psi[rt][k].y * ir);
          }
          a.T[r * 2] = (float)(tgt[rt].x * ir);
          a.T[r * 2 + 1] = (float)(tgt[rt].y * ir);
          a.S[r] = sflag[rt];
        }
      }
    }
    // ---- layer 1: h1[rt][kk] packs the outputs of tiles 2kk (slots 0..3) and 2kk+1 (slots 4..7)
    bf16x8 h1[2][8];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1f[t], xb[rt], acc, 0, 0, 0);
        const long r = row0 + 16 * rt + n;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int hid = 16 * t + 4 * g + i;
          const float z = acc[i] + b1s[hid];
          const float hv = silu(z);
          h1[rt][t >> 1][(t & 1) * 4 + i] = (bf16)hv;
          if (TRAIN && r < a.M) {
            a.Z1[r * H + hid] = z;
            a.H1[r * H + hid] = (bf16)hv;
          }
        }
      }
    }
    // ---- layer 2 and the layer-3 partial sums
    float part[2][2] = {{0.f, 0.f}, {0.f, 0.f}};
#pragma unroll 2
    for (int t2 = 0; t2 < 16; ++t2) {
      f32x4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const bf16x8 A = W2s[(t2 * 8 + kk) * 64 + lane];
        acc[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, h1[0][kk], acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, h1[1][kk], acc[1], 0, 0, 0);
      }
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        const long r = row0 + 16 * rt + n;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int hid = 16 * t2 + 4 * g + i;
          const float z = acc[rt][i] + b2s[hid];
          const float hv = bfr(silu(z));
          part[rt][0] = fmaf(W3s[hid], hv, part[rt][0]);
          part[rt][1] = fmaf(W3s[H + hid], hv, part[rt][1]);
          if (TRAIN && r < a.M) {
            a.Z2[r * H + hid] = z;
            a.H2[r * H + hid] = (bf16)hv;
          }
        }
      }
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        part[rt][o] += __shfl_xor(part[rt][o], 16, 64);
        part[rt][o] += __shfl_xor(part[rt][o], 32, 64);
      }
    if (g == 0) {
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        const long r = row0 + 16 * rt + n;
        if (r >= a.M) continue;
        const double sig = w.skip[16];
        const double n0 = (double)(part[rt][0] + b30), n1 = (double)(part[rt][1] + b31);
        const double* c = w.skip + sflag[rt] * 8;
        if (TRAIN) {
          // residual of the prediction in units of sigma, formed in FP64: (skip - target) / sigma + y
          const double ir = 1.0 / rho[rt];
          double l0 = -tgt[rt].x * ir, l1 = -tgt[rt].y * ir;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const double ur = psi[rt][k].x * ir, ui = psi[rt][k].y * ir;
            l0 += c[2 * k] * ur - c[2 * k + 1] * ui;
            l1 += c[2 * k] * ui + c[2 * k + 1] * ur;
          }
          a.out[r * 2] = (float)(l0 / sig + n0);
          a.out[r * 2 + 1] = (float)(l1 / sig + n1);
        } else {
          double g0 = rho[rt] * sig * n0, g1 = rho[rt] * sig * n1;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            g0 += c[2 * k] * psi[rt][k].x - c[2 * k + 1] * psi[rt][k].y;
            g1 += c[2 * k] * psi[rt][k].y + c[2 * k + 1] * psi[rt][k].x;
          }
          a.guess[r] = make_double2(g0, g1);
        }
      }
    }
  }
}

// C[m][n] = sum_k A(m, k) B(k, n) over k in [k_lo, k_hi), bf16 inputs with arbitrary strides,
// FP32 output. One wave per 16 x 16 tile of C; blockIdx.z selects a K slice whose partial goes to
// C + z * slice_stride (summed afterwards in fixed order).
__global__ __launch_bounds__(64) void gemm_bf16_kernel(const bf16* A, long sam, long sak, const bf16* B, long sbk, long sbn,
                                                       float* C, long scm, long scn, int Mo, int No, long K, long kslice,
                                                       long slice_stride) {
  const int lane = threadIdx.x, n = lane & 15, g = lane >> 4;
  const int tm = blockIdx.y, tn = blockIdx.x;
  const long k_lo = (long)blockIdx.z * kslice, k_hi = min(K, k_lo + kslice);
  const int am = tm * 16 + n, bn = tn * 16 + n;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (long k0 = k_lo; k0 < k_hi; k0 += 32) {
    bf16x8 av, bv;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const long k = k0 + 8 * g + j;
      const bool kin = k < k_hi;
      av[j] = (kin && am < Mo) ? A[am * sam + k * sak] : (bf16)0.0f;
      bv[j] = (kin && bn < No) ? B[k * sbk + bn * sbn] : (bf16)0.0f;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
  }
  float* Cz = C + (long)blockIdx.z * slice_stride;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = tm * 16 + 4 * g + i;
    if (m < Mo && bn < No) Cz[m * scm + bn * scn] = acc[i];
  }
}

// out[m * scm + n * scn] = sum_z part[z][m][n] (z ascending)
__global__ void sum_slices_kernel(const float* part, int nz, int Mo, int No, float* out, long scm, long scn) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)Mo * No) return;
  float s = 0.f;
  for (int z = 0; z < nz; ++z) s += part[(long)z * Mo * No + idx];
  out[(idx / No) * scm + (idx % No) * scn] = s;
}

// Column sums of an fp32 [M][N] matrix (N <= 256): pass 1 per chunk of rows, pass 2 in order.
__global__ void colsum_part_kernel(const float* X, long M, int N, long rows_per, float* part) {
  const int c = threadIdx.x;
  if (c >= N) return;
  const long r0 = (long)blockIdx.x * rows_per, r1 = min(M, r0 + rows_per);
  float s = 0.f;
  for (long r = r0; r < r1; ++r) s += X[r * N + c];
  part[(long)blockIdx.x * N + c] = s;
}
__global__ void colsum_final_kernel(const float* part, int nchunk, int N, float* out) {
  const int c = threadIdx.x;
  if (c >= N) return;
  float s = 0.f;
  for (int k = 0; k < nchunk; ++k) s += part[(long)k * N + c];
  out[c] = s;
}

// out holds the residual e / sigma of every row: L = mean |e / sigma|^2, dL/dy = 2 (e / sigma) / M.
__global__ __launch_bounds__(256) void loss_kernel(const float* out, long M, float* dY, bf16* dYb, double* part) {
  __shared__ double red[256];
  const float gscale = (float)(2.0 / (double)M);
  double loc = 0.0;
  for (long r = (long)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += (long)gridDim.x * blockDim.x) {
    const float e0 = out[2 * r], e1 = out[2 * r + 1];
    loc += (double)e0 * e0 + (double)e1 * e1;
    const float d0 = gscale * e0, d1 = gscale * e1;
    dY[2 * r] = d0;
    dY[2 * r + 1] = d1;
    dYb[2 * r] = (bf16)d0;
    dYb[2 * r + 1] = (bf16)d1;
  }
  red[threadIdx.x] = loc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void loss_final_kernel(const double* part, int nblk, double* loss_out, long M) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[b];
  *loss_out = s / (double)M;
}

// u_k = psi_{n-k} / rho and the target psi_{n+1} / rho of one raw training row.
__device__ inline int raw_row(const double* raw, long r, double tau, double2 (&u)[4], double2& t) {
  const double* p = raw + r * RAW;
  const double rho = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2] + p[3] * p[3] + tau * tau);
  const double ir = 1.0 / rho;
#pragma unroll
  for (int k = 0; k < 4; ++k) u[k] = make_double2(p[2 * k] * ir, p[2 * k + 1] * ir);
  t = make_double2(p[8] * ir, p[9] * ir);
  return p[12] != 0.0 ? 1 : 0;
}

// Per-block partials of G_s[k][l] = sum conj(u_k) u_l and r_s[k] = sum conj(u_k) t: [grid][2][20] complex.
constexpr int kGram = 2 * 20 * 2;
__global__ __launch_bounds__(256) void gram_kernel(const double* raw, long M, double tau, double* part) {
  __shared__ double red[256];
  double loc[kGram];
#pragma unroll
  for (int q = 0; q < kGram; ++q) loc[q] = 0.0;
  for (long r = (long)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += (long)gridDim.x * blockDim.x) {
    double2 u[4], t;
    const int s = raw_row(raw, r, tau, u, t);
#pragma unroll
    for (int sv = 0; sv < 2; ++sv) {
      if (s != sv) continue;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          double2 acc = make_double2(0.0, 0.0);
          tdde::dot_acc(acc, u[k], u[l]);
          loc[(sv * 20 + k * 4 + l) * 2] += acc.x;
          loc[(sv * 20 + k * 4 + l) * 2 + 1] += acc.y;
        }
        double2 acc = make_double2(0.0, 0.0);
        tdde::dot_acc(acc, u[k], t);
        loc[(sv * 20 + 16 + k) * 2] += acc.x;
        loc[(sv * 20 + 16 + k) * 2 + 1] += acc.y;
      }
    }
  }
  for (int q = 0; q < kGram; ++q) {
    red[threadIdx.x] = loc[q];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(long)blockIdx.x * kGram + q] = red[0];
    __syncthreads();
  }
}

// Sums the Gram partials in block order and solves G_s c_s = r_s (4x4 complex, partial pivoting).
__global__ void gram_solve_kernel(const double* part, int nblk, double* skip) {
  if (threadIdx.x != 0) return;
  for (int sv = 0; sv < 2; ++sv) {
    double2 A[4][5];
    for (int k = 0; k < 4; ++k)
      for (int l = 0; l < 5; ++l) {
        const int q = l < 4 ? sv * 20 + k * 4 + l : sv * 20 + 16 + k;
        double re = 0.0, im = 0.0;
        for (int b = 0; b < nblk; ++b) {
          re += part[(long)b * kGram + 2 * q];
          im += part[(long)b * kGram + 2 * q + 1];
        }
        A[k][l] = make_double2(re, im);
      }
    for (int col = 0; col < 4; ++col) {
      int pr = col;
      double best = 0.0;
      for (int r = col; r < 4; ++r) {
        const double v = A[r][col].x * A[r][col].x + A[r][col].y * A[r][col].y;
        if (v > best) { best = v; pr = r; }
      }
      for (int l = 0; l < 5; ++l) { const double2 tmp = A[col][l]; A[col][l] = A[pr][l]; A[pr][l] = tmp; }
      const double2 piv = A[col][col];
      const double pd = piv.x * piv.x + piv.y * piv.y;
      if (pd == 0.0) continue;
      for (int r = col + 1; r < 4; ++r) {
        // f = A[r][col] / piv
        const double2 f = make_double2((A[r][col].x * piv.x + A[r][col].y * piv.y) / pd,
                                       (A[r][col].y * piv.x - A[r][col].x * piv.y) / pd);
        for (int l = col; l < 5; ++l) {
          A[r][l].x -= f.x * A[col][l].x - f.y * A[col][l].y;
          A[r][l].y -= f.x * A[col][l].y + f.y * A[col][l].x;
        }
      }
    }
    double2 c[4];
    for (int k = 3; k >= 0; --k) {
      double2 v = A[k][4];
      for (int l = k + 1; l < 4; ++l) {
        v.x -= A[k][l].x * c[l].x - A[k][l].y * c[l].y;
        v.y -= A[k][l].x * c[l].y + A[k][l].y * c[l].x;
      }
      const double2 piv = A[k][k];
      const double pd = piv.x * piv.x + piv.y * piv.y;
      c[k] = pd > 0.0 ? make_double2((v.x * piv.x + v.y * piv.y) / pd, (v.y * piv.x - v.x * piv.y) / pd)
                      : make_double2(0.0, 0.0);
    }
    for (int k = 0; k < 4; ++k) {
      skip[sv * 8 + 2 * k] = c[k].x;
      skip[sv * 8 + 2 * k + 1] = c[k].y;
    }
  }
}

// Per-block partials of the squared residual |t - sum_k c[s][k] u_k|^2 of the fitted skip.
__global__ __launch_bounds__(256) void skip_resid_kernel(const double* raw, long M, double tau, const double* skip,
                                                         double* part) {
  __shared__ double red[256];
  double loc = 0.0;
  for (long r = (long)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += (long)gridDim.x * blockDim.x) {
    double2 u[4], t;
    const int s = raw_row(raw, r, tau, u, t);
    double e0 = t.x, e1 = t.y;
    for (int k = 0; k < 4; ++k) {
      const double cr = skip[s * 8 + 2 * k], ci = skip[s * 8 + 2 * k + 1];
      e0 -= cr * u[k].x - ci * u[k].y;
      e1 -= cr * u[k].y + ci * u[k].x;
    }
    loc += e0 * e0 + e1 * e1;
  }
  red[threadIdx.x] = loc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void skip_sigma_kernel(const double* part, int nblk, long M, double* skip) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[b];
  skip[16] = fmax(sqrt(s / (double)M), 1e-300);
}

// dZ2 = (dY W3) * silu'(Z2)  (in place over Z2, plus a bf16 copy)
__global__ void dz2_kernel(const float* dY, const float* W3r, float* Z2, bf16* dZ2b, long M) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * H) return;
  const long r = idx / H;
  const int h = (int)(idx - r * H);
  const float d = (dY[2 * r] * W3r[h] + dY[2 * r + 1] * W3r[H + h]) * dsilu(Z2[idx]);
  Z2[idx] = d;
  dZ2b[idx] = (bf16)d;
}

// dZ1 = dH1 * silu'(Z1)  (in place over Z1, plus a bf16 copy)
__global__ void dz1_kernel(const float* dH1, float* Z1, bf16* dZ1b, long M) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * H) return;
  const float d = dH1[idx] * dsilu(Z1[idx]);
  Z1[idx] = d;
  dZ1b[idx] = (bf16)d;
}

__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int n, float lr, float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
}

// BF16 copies of the weights: W1, W2 (plain and permuted for the fused forward), W3 rounded.
__global__ void refresh_kernel(const float* P, bf16* W1b, bf16* W2b, bf16* W2p, float* W3r) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < H * F) W1b[idx] = (bf16)P[OFF_W1 + idx];
  if (idx < H * H) {
    W2b[idx] = (bf16)P[OFF_W2 + idx];
    // permuted: idx = ((t2 * 8 + kk) * 64 + l) * 8 + j
    const int j = idx & 7, l = (idx >> 3) & 63, kk = (idx >> 9) & 7, t2 = idx >> 12;
    const int row = 16 * t2 + (l & 15);
    const int col = 16 * (2 * kk + (j >> 2)) + 4 * (l >> 4) + (j & 3);
    W2p[idx] = (bf16)P[OFF_W2 + row * H + col];
  }
  if (idx < 2 * H) W3r[idx] = (float)(bf16)P[OFF_W3 + idx];
}

}  // namespace

struct tdde_mlp {
  hipStream_t stream = nullptr;
  std::string err;
  int Mcap = 0;
  double tau = 1e-6;
  long step = 0;
  std::vector<void*> allocs;
  float *P = nullptr, *G = nullptr, *Mm = nullptr, *Vv = nullptr;
  bf16 *W1b = nullptr, *W2b = nullptr, *W2p = nullptr;
  float* W3r = nullptr;
  double* skip = nullptr;
  // scratch
  float *out = nullptr, *Z1 = nullptr, *Z2 = nullptr, *U = nullptr, *T = nullptr, *dY = nullptr, *dH = nullptr;
  bf16 *H1 = nullptr, *H2 = nullptr, *X = nullptr, *dYb = nullptr, *dZb = nullptr;
  int* S = nullptr;
  float* gpart = nullptr;     // split-K partials
  double* lpart = nullptr;    // loss partials
  double* loss_dev = nullptr;
  float* cpart = nullptr;     // colsum partials
  PulseDev* pulses = nullptr;
  int pulse_batch = 0, pulse_nf = 0;
};

namespace {

constexpr int kLossBlocks = 256;
constexpr long kSliceK = 2048;
constexpr long kColRows = 512;

#define MLP_TRY(m, call)                                                          \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      (m)->err = std::string(#call) + ": " + hipGetErrorString(e_);               \
      return TDDE_ERR_HIP;                                                        \
    }                                                                             \
  } while (0)

template <typename X> tdde_status mlp_alloc(tdde_mlp* m, X** p, size_t n) {
  void* q = nullptr;
  if (hipMalloc(&q, (n ? n : 1) * sizeof(X)) != hipSuccess) {
    m->err = "hipMalloc failed";
    return TDDE_ERR_NOMEM;
  }
  m->allocs.push_back(q);
  *p = static_cast<X*>(q);
  return TDDE_OK;
}

Weights weights_of(const tdde_mlp* m) {
  Weights w;
  w.W1 = m->W1b;
  w.W2p = reinterpret_cast<const bf16x8*>(m->W2p);
  w.P = m->P;
  w.W3r = m->W3r;
  w.skip = m->skip;
  return w;
}

int fwd_grid(long M) {
  const long passes = (M + 31) / 32;
  long blocks = (passes + 3) / 4;
  return (int)std::max(1L, std::min(blocks, 1024L));
}

tdde_status gemm(tdde_mlp* m, const bf16* A, long sam, long sak, const bf16* B, long sbk, long sbn, float* C, long scm,
                 long scn, int Mo, int No, long K) {
  const int nz = (int)std::max(1L, (K + kSliceK - 1) / kSliceK);
  dim3 grid((No + 15) / 16, (Mo + 15) / 16, nz);
  if (nz == 1) {
    hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(64), 0, m->stream, A, sam, sak, B, sbk, sbn, C, scm, scn, Mo, No, K,
                       kSliceK, 0L);
  } else {
    if ((long)nz * Mo * No > (long)(m->Mcap / kSliceK + 2) * H * H) {
      m->err = "split-K scratch too small";
      return TDDE_ERR_ARG;
    }
    hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(64), 0, m->stream, A, sam, sak, B, sbk, sbn, m->gpart, (long)No, 1L,
                       Mo, No, K, kSliceK, (long)Mo * No);
    hipLaunchKernelGGL(sum_slices_kernel, dim3(((long)Mo * No + 255) / 256), dim3(256), 0, m->stream, m->gpart, nz, Mo, No,
                       C, scm, scn);
  }
  MLP_TRY(m, hipGetLastError());
  return TDDE_OK;
}

tdde_status colsum(tdde_mlp* m, const float* X, long M, int N, float* out) {
  const int nchunk = (int)std::max(1L, (M + kColRows - 1) / kColRows);
  hipLaunchKernelGGL(colsum_part_kernel, dim3(nchunk), dim3(256), 0, m->stream, X, M, N, kColRows, m->cpart);
  hipLaunchKernelGGL(colsum_final_kernel, dim3(1), dim3(256), 0, m->stream, m->cpart, nchunk, N, out);
  MLP_TRY(m, hipGetLastError());
  return TDDE_OK;
}

tdde_status refresh(tdde_mlp* m) {
  hipLaunchKernelGGL(refresh_kernel, dim3((H * H + 255) / 256), dim3(256), 0, m->stream, m->P, m->W1b, m->W2b, m->W2p,
                     m->W3r);
  MLP_TRY(m, hipGetLastError());
  return TDDE_OK;
}

FwdArgs train_args(tdde_mlp* m, const double* raw, long M) {
  FwdArgs a{};
  a.M = M;
  a.tau = m->tau;
  a.raw = raw;
  a.out = m->out;
  a.Z1 = m->Z1;
  a.Z2 = m->Z2;
  a.H1 = m->H1;
  a.H2 = m->H2;
  a.X = m->X;
  a.U = m->U;
  a.T = m->T;
  a.S = m->S;
  return a;
}

}  // namespace

int64_t tdde_mlp_param_count(void) { return N_PARAM; }

const char* tdde_mlp_last_error(const tdde_mlp* m) { return m ? m->err.c_str() : "null network"; }

tdde_status tdde_mlp_create(int32_t train_rows, double tau, void* stream, tdde_mlp** out) {
  if (!out || train_rows <= 0 || !(tau > 0.0)) return TDDE_ERR_ARG;
  *out = nullptr;
  tdde_mlp* m = new tdde_mlp();
  m->stream = static_cast<hipStream_t>(stream);
  m->Mcap = train_rows;
  m->tau = tau;
  const size_t M = (size_t)train_rows;
  tdde_status s;
#define ALLOC(ptr, n) \
  if ((s = mlp_alloc(m, &ptr, n)) != TDDE_OK) { tdde_mlp_destroy(m); return s; }
  ALLOC(m->P, N_PARAM);
  ALLOC(m->G, N_PARAM);
  ALLOC(m->Mm, N_PARAM);
  ALLOC(m->Vv, N_PARAM);
  ALLOC(m->W1b, H * F);
  ALLOC(m->W2b, H * H);
  ALLOC(m->W2p, H * H);
  ALLOC(m->W3r, 2 * H);
  ALLOC(m->out, 2 * M);
  ALLOC(m->Z1, M * H);
  ALLOC(m->Z2, M * H);
  ALLOC(m->dH, M * H);
  ALLOC(m->U, 8 * M);
  ALLOC(m->T, 2 * M);
  ALLOC(m->dY, 2 * M);
  ALLOC(m->H1, M * H);
  ALLOC(m->H2, M * H);
  ALLOC(m->X, M * F);
  ALLOC(m->dYb, 2 * M);
  ALLOC(m->dZb, M * H);
  ALLOC(m->S, M);
  ALLOC(m->gpart, (size_t)(M / kSliceK + 2) * H * H);
  ALLOC(m->lpart, (size_t)kLossBlocks * kGram);
  ALLOC(m->skip, N_SKIP);
  ALLOC(m->loss_dev, 1);
  ALLOC(m->cpart, (size_t)((M + kColRows - 1) / kColRows + 1) * H);
#undef ALLOC
  if (hipMemset(m->P, 0, N_PARAM * sizeof(float)) != hipSuccess || hipMemset(m->Mm, 0, N_PARAM * sizeof(float)) != hipSuccess ||
      hipMemset(m->Vv, 0, N_PARAM * sizeof(float)) != hipSuccess || hipMemset(m->G, 0, N_PARAM * sizeof(float)) != hipSuccess) {
    tdde_mlp_destroy(m);
    return TDDE_ERR_HIP;
  }
  {
    double sk[N_SKIP] = {0};
    sk[0] = sk[8] = 1.0;  // previous-state predictor until a fit or set_skip
    sk[16] = 1.0;
    if (hipMemcpy(m->skip, sk, sizeof(sk), hipMemcpyHostToDevice) != hipSuccess) {
      tdde_mlp_destroy(m);
      return TDDE_ERR_HIP;
    }
  }
  if (refresh(m) != TDDE_OK || hipDeviceSynchronize() != hipSuccess) {
    tdde_mlp_destroy(m);
    return TDDE_ERR_HIP;
  }
  *out = m;
  return TDDE_OK;
}

tdde_status tdde_mlp_destroy(tdde_mlp* m) {
  if (!m) return TDDE_OK;
  for (void* p : m->allocs) (void)hipFree(p);
  delete m;
  return TDDE_OK;
}

tdde_status tdde_mlp_set_params(tdde_mlp* m, const float* host) {
  if (!m || !host) return TDDE_ERR_ARG;
  MLP_TRY(m, hipMemcpyAsync(m->P, host, N_PARAM * sizeof(float), hipMemcpyHostToDevice, m->stream));
  MLP_TRY(m, hipMemsetAsync(m->Mm, 0, N_PARAM * sizeof(float), m->stream));
  MLP_TRY(m, hipMemsetAsync(m->Vv, 0, N_PARAM * sizeof(float), m->stream));
  m->step = 0;
  tdde_status s = refresh(m);
  if (s != TDDE_OK) return s;
  MLP_TRY(m, hipStreamSynchronize(m->stream));
  return TDDE_OK;
}

tdde_status tdde_mlp_get_params(tdde_mlp* m, float* host) {
  if (!m || !host) return TDDE_ERR_ARG;
  MLP_TRY(m, hipMemcpyAsync(host, m->P, N_PARAM * sizeof(float), hipMemcpyDeviceToHost, m->stream));
  MLP_TRY(m, hipStreamSynchronize(m->stream));
  return TDDE_OK;
}

tdde_status tdde_mlp_get_grads(tdde_mlp* m, float* host) {
  if (!m || !host) return TDDE_ERR_ARG;
  MLP_TRY(m, hipMemcpyAsync(host, m->G, N_PARAM * sizeof(float), hipMemcpyDeviceToHost, m->stream));
  MLP_TRY(m, hipStreamSynchronize(m->stream));
  return TDDE_OK;
}

tdde_status tdde_mlp_forward(tdde_mlp* m, const double* raw, int32_t M, float* out) {
  if (!m || !raw || !out || M <= 0 || M > m->Mcap) return TDDE_ERR_ARG;
  FwdArgs a = train_args(m, raw, M);
  hipLaunchKernelGGL(mlp_fwd_kernel<true>, dim3(fwd_grid(M)), dim3(256), 0, m->stream, weights_of(m), a);
  MLP_TRY(m, hipGetLastError());
  MLP_TRY(m, hipMemcpyAsync(out, m->out, (size_t)M * 2 * sizeof(float), hipMemcpyDeviceToDevice, m->stream));
  return TDDE_OK;
}

tdde_status tdde_mlp_backward(tdde_mlp* m, const double* raw, int32_t Mi, double* loss) {
  if (!m || !raw || Mi <= 0 || Mi > m->Mcap) return TDDE_ERR_ARG;
  const long M = Mi;
  FwdArgs a = train_args(m, raw, M);
  hipLaunchKernelGGL(mlp_fwd_kernel<true>, dim3(fwd_grid(M)), dim3(256), 0, m->stream, weights_of(m), a);
  MLP_TRY(m, hipGetLastError());
  hipLaunchKernelGGL(loss_kernel, dim3(kLossBlocks), dim3(256), 0, m->stream, m->out, M, m->dY, m->dYb, m->lpart);
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(64), 0, m->stream, m->lpart, kLossBlocks, m->loss_dev, M);
  MLP_TRY(m, hipGetLastError());
  tdde_status s;
  // layer 3: dW3 = dY^T H2, db3 = colsum(dY)
  if ((s = gemm(m, m->dYb, 1, 2, m->H2, H, 1, m->G + OFF_W3, H, 1, 2, H, M)) != TDDE_OK) return s;
  if ((s = colsum(m, m->dY, M, 2, m->G + OFF_B3)) != TDDE_OK) return s;
  // dZ2 = (dY W3) silu'(Z2)
  hipLaunchKernelGGL(dz2_kernel, dim3((M * H + 255) / 256), dim3(256), 0, m->stream, m->dY, m->W3r, m->Z2, m->dZb, M);
  MLP_TRY(m, hipGetLastError());
  // layer 2: dW2 = dZ2^T H1, db2 = colsum(dZ2), dH1 = dZ2 W2
  if ((s = gemm(m, m->dZb, 1, H, m->H1, H, 1, m->G + OFF_W2, H, 1, H, H, M)) != TDDE_OK) return s;
  if ((s = colsum(m, m->Z2, M, H, m->G + OFF_B2)) != TDDE_OK) return s;
  if ((s = gemm(m, m->dZb, H, 1, m->W2b, H, 1, m->dH, H, 1, (int)M, H, H)) != TDDE_OK) return s;
  // dZ1 = dH1 silu'(Z1); layer 1: dW1 = dZ1^T X, db1 = colsum(dZ1)
  hipLaunchKernelGGL(dz1_kernel, dim3((M * H + 255) / 256), dim3(256), 0, m->stream, m->dH, m->Z1, m->dZb, M);
  MLP_TRY(m, hipGetLastError());
  if ((s = gemm(m, m->dZb, 1, H, m->X, F, 1, m->G + OFF_W1, F, 1, H, F, M)) != TDDE_OK) return s;
  if ((s = colsum(m, m->Z1, M, H, m->G + OFF_B1)) != TDDE_OK) return s;
  if (loss) {
    MLP_TRY(m, hipMemcpyAsync(loss, m->loss_dev, sizeof(double), hipMemcpyDeviceToHost, m->stream));
    MLP_TRY(m, hipStreamSynchronize(m->stream));
  }
  return TDDE_OK;
}

tdde_status tdde_mlp_adam(tdde_mlp* m, float lr) {
  if (!m || !(lr > 0.f)) return TDDE_ERR_ARG;
  m->step++;
  const float bc1 = 1.0f - std::pow(0.9f, (float)m->step), bc2 = 1.0f - std::pow(0.999f, (float)m->step);
  hipLaunchKernelGGL(adam_kernel, dim3((N_PARAM + 255) / 256), dim3(256), 0, m->stream, m->P, m->G, m->Mm, m->Vv, N_PARAM,
                     lr, bc1, bc2);
  MLP_TRY(m, hipGetLastError());
  return refresh(m);
}

tdde_status tdde_mlp_fit_skip(tdde_mlp* m, const double* raw, int32_t M) {
  if (!m || !raw || M <= 0) return TDDE_ERR_ARG;
  hipLaunchKernelGGL(gram_kernel, dim3(kLossBlocks), dim3(256), 0, m->stream, raw, (long)M, m->tau, m->lpart);
  hipLaunchKernelGGL(gram_solve_kernel, dim3(1), dim3(64), 0, m->stream, (const double*)m->lpart, kLossBlocks, m->skip);
  hipLaunchKernelGGL(skip_resid_kernel, dim3(kLossBlocks), dim3(256), 0, m->stream, raw, (long)M, m->tau,
                     (const double*)m->skip, m->lpart);
  hipLaunchKernelGGL(skip_sigma_kernel, dim3(1), dim3(64), 0, m->stream, (const double*)m->lpart, kLossBlocks, (long)M,
                     m->skip);
  MLP_TRY(m, hipGetLastError());
  MLP_TRY(m, hipStreamSynchronize(m->stream));
  return TDDE_OK;
}

tdde_status tdde_mlp_set_skip(tdde_mlp* m, const double* c, double sigma) {
  if (!m || !c || !(sigma >= 0.0)) return TDDE_ERR_ARG;
  double sk[N_SKIP];
  std::memcpy(sk, c, 16 * sizeof(double));
  sk[16] = sigma;
  MLP_TRY(m, hipMemcpyAsync(m->skip, sk, sizeof(sk), hipMemcpyHostToDevice, m->stream));
  MLP_TRY(m, hipStreamSynchronize(m->stream));
  return TDDE_OK;
}

tdde_status tdde_mlp_get_skip(tdde_mlp* m, double* c, double* sigma) {
  if (!m || !c || !sigma) return TDDE_ERR_ARG;
  double sk[N_SKIP];
  MLP_TRY(m, hipMemcpyAsync(sk, m->skip, sizeof(sk), hipMemcpyDeviceToHost, m->stream));
  MLP_TRY(m, hipStreamSynchronize(m->stream));
  std::memcpy(c, sk, 16 * sizeof(double));
  *sigma = sk[16];
  return TDDE_OK;
}

tdde_status tdde_mlp_set_pulses(tdde_mlp* m, const tdde_pulse* p, int32_t batch, int32_t nf) {
  if (!m || !p || batch <= 0 || nf <= 0) return TDDE_ERR_ARG;
  if (batch * nf > m->pulse_batch * m->pulse_nf) {
    tdde_status s = mlp_alloc(m, &m->pulses, (size_t)batch * nf);
    if (s != TDDE_OK) return s;
  }
  std::vector<PulseDev> h((size_t)batch * nf);
  for (size_t i = 0; i < h.size(); ++i) h[i] = PulseDev{p[i].amp, p[i].T, p[i].omega, p[i].phase, p[i].envelope, 0};
  MLP_TRY(m, hipMemcpy(m->pulses, h.data(), h.size() * sizeof(PulseDev), hipMemcpyHostToDevice));
  m->pulse_batch = batch;
  m->pulse_nf = nf;
  return TDDE_OK;
}

tdde_status tdde_mlp_guess(tdde_mlp* m, const void* const hist[4], int32_t batch, int64_t E, int32_t nr, double t_n,
                           double dt, void* guess_out) {
  if (!m || !hist || !guess_out || batch <= 0 || E <= 0 || nr <= 0 || E % (2 * nr) != 0) return TDDE_ERR_ARG;
  for (int k = 0; k < 4; ++k)
    if (!hist[k] || hist[k] == guess_out) return TDDE_ERR_ARG;
  if (!m->pulses || batch != m->pulse_batch) {
    m->err = "set_pulses with the same batch first";
    return TDDE_ERR_STATE;
  }
  FwdArgs a{};
  a.M = (long)batch * E;
  a.tau = m->tau;
  a.hist0 = (const double2*)hist[0];
  a.hist1 = (const double2*)hist[1];
  a.hist2 = (const double2*)hist[2];
  a.hist3 = (const double2*)hist[3];
  a.E = E;
  a.nr = nr;
  a.n_fields = m->pulse_nf;
  a.pulses = m->pulses;
  a.t_n = t_n;
  a.dt = dt;
  a.guess = (double2*)guess_out;
  hipLaunchKernelGGL(mlp_fwd_kernel<false>, dim3(fwd_grid(a.M)), dim3(256), 0, m->stream, weights_of(m), a);
  MLP_TRY(m, hipGetLastError());
  return TDDE_OK;
}
