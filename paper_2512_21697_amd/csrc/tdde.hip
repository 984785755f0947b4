// Host side of the TDDE library: context, operator upload, preconditioner factorisation and the
// C ABI declared in include/tdde.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <iterator>

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <cstddef>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tdde.h"
#include "solver.hpp"
#include "split.hpp"

using namespace tdde;
using cd = std::complex<double>;

// Most persistent work-groups placed on one CU (the default launch shape).
constexpr int kMaxWgPerCu = 4;

struct tdde_ctx {
  tdde_dims d{};
  hipStream_t stream = nullptr;
  std::string err;
  int E = 0;            // unknowns per instance
  bool assembled = false;
  bool dt_set = false;
  bool field_set = false;
  bool pulses_set = false;
  bool use_table = false;   // field table (tdde_set_field_table) instead of the pulses
  double* ftab = nullptr;
  int ftab_rows = 0;
  size_t ftab_cap = 0;
  double dt = 0.0;
  std::vector<void*> allocs;
  // host copy of what the preconditioner needs
  std::vector<double> kappa, h_poly, h_chan, s_poly;
  int n_h = 0, n_s = 0, has_chan = 0;
  // device operator
  DevOp<double> op64{};
  DevOp<float> op32{};
  DevPrec<double> pc64{};
  DevPrec<float> pc32{};
  std::vector<int> block_of;
  int nblk = 0;
  bool prec_alloc = false;
  int seg_min = 24;              // least rows per preconditioner segment (tdde_set_prec_segment)
  // graph mode (tdde_set_graph): the launch sequence of a persistent chunk (two fill kernels and the
  // cooperative solver launch) captured once per kernel variant and grid, replayed with the chunk's
  // arguments written into the captured kernel nodes
  bool use_graph = false;
  struct Captured {
    int v = -1, n_wg = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t solver = nullptr, zero_cnt = nullptr;
  } cap;
  size_t cap_lu = 0, cap_t = 0;  // allocated factor / boundary-matrix elements
  size_t order_cap = 0;          // ints of the chain-order buffer
  // workspace
  KVec<double> v64{};
  KVec<float> v32{};
  KVec<double> v64np{};  // aliases without preconditioner (p^ = p, s^ = s)
  KVec<float> v32np{};
  double2* bvec = nullptr;
  double2* bvec2 = nullptr;
  double2* xalt = nullptr;  // second iterate buffer (x + alpha p^ formed ahead of the half-step test)
  double2* r64 = nullptr;
  float2* rhs32 = nullptr;
  double2* part = nullptr;
  unsigned* bar = nullptr;
  int* counters = nullptr;
  int n_counters = 0;
  StatsDev* stats_dev = nullptr;
  int stats_cap = 0;
  double* fvals = nullptr;
  PulseDev* pulses = nullptr;
  int* n_steps_dev = nullptr;
  int n_wg = 0, G = 0;          // grid of the variant in use (set per launch)
  int var_wg[4] = {0, 0, 0, 0};  // co-resident work-groups of each persistent-kernel variant
  int var_occ[4] = {0, 0, 0, 0}; // occupancy limit (work-groups per CU) of each variant
  int ncu = 0;
  unsigned long long* marks = nullptr;
  int n_marks = 0;
  const double2* shadow = nullptr;  // test hook: shadow residual of the first BiCGSTAB cycle of a solve
  // photoelectron spectrum (tdde_spectrum_setup)
  bool spec_set = false;
  int spec_nblk = 0, spec_maxlev = 0, spec_ngrid = 0;
  int* spec_blk_of = nullptr;     // [nang] eigen-block of every channel
  int* spec_lev0 = nullptr;       // [nblk + 1] first level of every block
  double* spec_E = nullptr;       // [total levels + 2 nblk]: per block the level below, its levels, the level above
  double* spec_U = nullptr;       // [total levels][2][nr] S v_n
  double* spec_grid = nullptr;    // [n_grid]
  double* spec_dens = nullptr;    // [batch][nang][max levels]
  double* spec_err = nullptr;     // [batch]
  // kernel-per-window solver (tdde_set_split)
  bool split = false;
  bool prec_f32 = false;          // FP32 preconditioner factors in the kernel-per-window solver
  int sp_G = 0;                   // work-groups per instance of its apply and vector kernels
  SplitCtl* sp_ctl = nullptr;     // [batch] control blocks
  int* sp_cnt = nullptr;          // [batch][kSpCntLine] arrival counters
  double2* sp_part = nullptr;     // [batch][sp_G][kSpSlots]
  int* sp_flag = nullptr;         // pinned host memory [2]: unfinished instances after a block
  hipEvent_t sp_ev[2] = {nullptr, nullptr};
  std::vector<int> ones;          // n_steps of a single step
  std::vector<hipEvent_t> sp_tev; // timing events of the apply kernel (tdde_debug_split_timing): pairs
  int sp_tcap = 0, sp_tn = 0;     // pairs enabled, pairs recorded
};

// persistent kernel variants, index = 2 * mixed + preconditioned (each compiled in its own object
// from persistent.hip)
namespace tdde {
const void* persistent_variant_0();
const void* persistent_variant_1();
const void* persistent_variant_2();
const void* persistent_variant_3();
}  // namespace tdde
static const void* persistent_variant(int idx) {
  switch (idx) {
    case 0: return persistent_variant_0();
    case 1: return persistent_variant_1();
    case 2: return persistent_variant_2();
    default: return persistent_variant_3();
  }
}

static std::string g_create_err;

// ------------------------------------------------------------------------------------------ static scratch
// Device array behind tdde_solve_static (the entry point for callers that cannot allocate): the
// solve's scratch lives here instead of in the context's workspace. Every GPU holds its own copy
// from module load until the process ends. In host code `scratch` is only a host-side stand-in;
// its device address comes from hipGetSymbolAddress, resolved once per device in tdde_create
// (with that device current) and kept in g_scratch_dev.
static __device__ __align__(256) unsigned char scratch[TDDE_STATIC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static void* g_scratch_dev[kMaxDevices] = {};
static hipError_t g_scratch_err[kMaxDevices] = {};
static bool g_scratch_done[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// Resolve the current device's copy of `scratch` (first call on a device only).
static void resolve_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_done[dev]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  g_scratch_err[dev] = e;
  g_scratch_dev[dev] = e == hipSuccess ? ptr : nullptr;
  g_scratch_done[dev] = true;
}

#define HIP_TRY(ctx, call)                                                                    \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      (ctx)->err = std::string(#call) + ": " + hipGetErrorString(e_);                         \
      return TDDE_ERR_HIP;                                                                    \
    }                                                                                         \
  } while (0)

static tdde_status fail(tdde_ctx* c, tdde_status s, const std::string& m) {
  if (c) c->err = m;
  return s;
}

template <typename X> static tdde_status dev_alloc(tdde_ctx* c, X** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(X));
  if (e != hipSuccess) {
    c->err = std::string("hipMalloc: ") + hipGetErrorString(e);
    return TDDE_ERR_NOMEM;
  }
  c->allocs.push_back(q);
  *p = static_cast<X*>(q);
  return TDDE_OK;
}

template <typename X> static tdde_status upload(tdde_ctx* c, X** p, const X* h, size_t count) {
  tdde_status s = dev_alloc(c, p, count);
  if (s != TDDE_OK) return s;
  if (count) HIP_TRY(c, hipMemcpy(*p, h, count * sizeof(X), hipMemcpyHostToDevice));
  return TDDE_OK;
}

template <typename X> static std::vector<float> to_f32(const X* p, size_t n) {
  std::vector<float> o(n);
  for (size_t i = 0; i < n; ++i) o[i] = (float)p[i];
  return o;
}

// ------------------------------------------------------------------------------------------ kernels

__global__ void zero_words(unsigned* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void apply_kernel(DevOp<T> op, const c2_t<T>* x, c2_t<T>* y, double2 as,
                                                         double2 ah, const double* fvals, int n_fields, int E, int B) {
  __shared__ TileLds<T> L;
  __shared__ TermLds tl;
  // work-group w: instance b = (w / 8) % B, tile t = (w / (8 B)) * 8 + w % 8, so tile t of every
  // instance runs on XCD t % 8 (tile_coords: all channels of a radial tile on one XCD; the
  // instances of a tile close together, operator bands reused from that XCD's L2)
  const int w = blockIdx.x;
  const int b = (w >> 3) % B;
  const int t = (w / (8 * B)) * 8 + (w & 7);
  if (t >= op.nang * op.n_itiles) return;  // uniform over the work-group
  int j, it;
  tile_coords(op.nang, op.n_itiles, t, j, it);
  terms_to_lds<T>(op, tl, [&](int m) { return fvals[(size_t)b * n_fields + op.t_field[m]]; });
  const c2_t<T>* xb = x + (size_t)b * E;
  SH<T> r = apply_tile<T, false, kGatherBatch, 1>(op, xb, j, it * kTileR, tl, L);
  const long e = tile_elem(op.nr, j, it);
  if (e >= 0) {
    c2_t<T> out = cmul<T>(to_c<T>(as), r.sx);
    out = cfma<T>(to_c<T>(ah), r.hx, out);
    y[(size_t)b * E + e] = out;
  }
}

template <typename T>
// two work-groups per CU: the chain solve fits 256 registers per lane without spills
__global__ __launch_bounds__(kThreads, 2) void precond_kernel(DevPrec<T> pc, int nr, const c2_t<T>* in, c2_t<T>* out, int E) {
  __shared__ ChainLds<T> lds;
  const int b = blockIdx.y;
  const int* js = nullptr;
  const int nk = chain_item(pc, blockIdx.x, js);
  if (nk == 0) return;  // padding item (uniform over the work-group)
  const size_t ib = (size_t)b * E;
  ChainIO<T> io;
  io.r = nullptr;
  io.v = nullptr;
  io.pz = const_cast<c2_t<T>*>(in) + ib;
  io.out = out + ib;
  io.c1 = io.c2 = make_double2(0, 0);
  chain_solve<T, MODE_IN>(pc, pc.block_of[js[0]], nr, io, js, nk, lds);
}

// ------------------------------------------------------------------------------------------ helpers

static int band_index(int hb, int nr, int s, int s2, int d, int i) {
  return ((s * 2 + s2) * (2 * hb + 1) + (d + hb)) * nr + i;
}

static bool any_offdiag(const double* bands, int count, int hb, int nr, int stride_complex) {
  // bands: count blocks of [2][2][nb][nr] (x stride_complex doubles per value)
  const size_t blk = (size_t)(2 * hb + 1) * nr * stride_complex;
  for (int c = 0; c < count; ++c)
    for (int sel = 1; sel <= 2; ++sel) {
      const double* p = bands + ((size_t)c * 4 + sel) * blk;
      for (size_t k = 0; k < blk; ++k)
        if (p[k] != 0.0) return true;
    }
  return false;
}

// ------------------------------------------------------------------------------------------ C ABI
// (the declarations in tdde.h give every entry point C linkage)

const char* tdde_status_string(tdde_status s) {
  switch (s) {
    case TDDE_OK: return "ok";
    case TDDE_NOT_CONVERGED: return "not converged";
    case TDDE_BREAKDOWN: return "breakdown";
    case TDDE_NONFINITE: return "non-finite value";
    case TDDE_ERR_ARG: return "invalid argument";
    case TDDE_ERR_HIP: return "HIP error";
    case TDDE_ERR_NOMEM: return "out of device memory";
    case TDDE_ERR_STATE: return "invalid call order";
  }
  return "unknown status";
}

const char* tdde_last_error(const tdde_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

tdde_status tdde_create(const tdde_dims* dims, void* hip_stream, tdde_ctx** out) {
  if (!dims || !out) { g_create_err = "null argument"; return TDDE_ERR_ARG; }
  *out = nullptr;
  if (dims->nr <= 0 || dims->nang <= 0 || dims->half_band != kHB || dims->batch <= 0 || dims->n_fields <= 0 ||
      dims->n_fields > kMaxFields) {
    g_create_err = "dims out of range (nr, nang, batch > 0; half_band == 6; 1 <= n_fields <= 16)";
    return TDDE_ERR_ARG;
  }
  if ((double)dims->nr * dims->nang * 2 > 2.0e9) { g_create_err = "instance too large"; return TDDE_ERR_ARG; }
  resolve_scratch();
  tdde_ctx* c = new tdde_ctx();
  c->d = *dims;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->E = dims->nang * 2 * dims->nr;
  *out = c;
  return TDDE_OK;
}

tdde_status tdde_destroy(tdde_ctx* ctx) {
  if (!ctx) return TDDE_OK;
  if (ctx->cap.exec) (void)hipGraphExecDestroy(ctx->cap.exec);
  if (ctx->cap.graph) (void)hipGraphDestroy(ctx->cap.graph);
  for (hipEvent_t e : ctx->sp_ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->sp_tev) (void)hipEventDestroy(e);
  if (ctx->sp_flag) (void)hipHostFree(ctx->sp_flag);
  for (void* p : ctx->allocs) (void)hipFree(p);
  delete ctx;
  return TDDE_OK;
}

template <typename T>
static tdde_status build_devop(tdde_ctx* c, const tdde_operator_desc* o, DevOp<T>& op, const std::vector<double>& tval,
                               const std::vector<int>& rowptr_abs, const std::vector<int>& mask) {
  const int nr = c->d.nr, nang = c->d.nang, hb = c->d.half_band, nb = 2 * hb + 1;
  const size_t bsz = (size_t)4 * nb * nr;
  op.nr = nr; op.nang = nang; op.hb = hb; op.nb = nb;
  op.n_h = o->n_h; op.n_s = o->n_s; op.has_chan = o->h_chan != nullptr;
  op.n_terms = o->n_terms;
  op.n_itiles = (nr + kTileR - 1) / kTileR;
  op.pq_h = o->n_h > 0 && any_offdiag(o->h_poly, o->n_h, hb, nr, 1);
  op.pq_s = o->n_s > 0 && any_offdiag(o->s_poly, o->n_s, hb, nr, 1);
  op.pq_chan = op.has_chan && any_offdiag(o->h_chan, nang, hb, nr, 2);
  const int64_t nnz = o->n_terms ? o->a_off[o->n_terms] : 0;
  auto up = [&](auto** dst, const double* src, size_t n) -> tdde_status {
    using X = std::remove_pointer_t<std::remove_reference_t<decltype(*dst)>>;
    if constexpr (std::is_same<X, const double>::value || std::is_same<X, double>::value) {
      return upload(c, (double**)dst, src, n);
    } else {
      std::vector<float> f = to_f32(src, n);
      return upload(c, (float**)dst, f.data(), n);
    }
  };
  tdde_status s;
  // H0 and S per distinct kappa: the kappa polynomials summed (Horner) on the host
  {
    std::map<double, int> seen;
    std::vector<int> kblk(nang);
    std::vector<double> kvals;
    for (int j = 0; j < nang; ++j) {
      auto it = seen.find(o->kappa[j]);
      if (it == seen.end()) {
        it = seen.emplace(o->kappa[j], (int)kvals.size()).first;
        kvals.push_back(o->kappa[j]);
      }
      kblk[j] = it->second;
    }
    const int nkb = (int)kvals.size();
    auto sum_poly = [&](const double* poly, int npoly, std::vector<double>& outv) {
      outv.assign((size_t)nkb * bsz, 0.0);
      for (int kb = 0; kb < nkb; ++kb) {
        const double kap = kvals[kb];
        double* dst = outv.data() + (size_t)kb * bsz;
        for (size_t e = 0; e < bsz; ++e) {
          double acc = poly[(size_t)(npoly - 1) * bsz + e];
          for (int n = npoly - 2; n >= 0; --n) acc = std::fma(acc, kap, poly[(size_t)n * bsz + e]);
          dst[e] = acc;
        }
      }
    };
    if ((s = upload(c, (int**)&op.kblk_of, kblk.data(), kblk.size())) != TDDE_OK) return s;
    std::vector<double> blk;
    op.h_blk = nullptr;
    op.s_blk = nullptr;
    if (o->n_h > 0) {
      sum_poly(o->h_poly, o->n_h, blk);
      if ((s = up((T**)&op.h_blk, blk.data(), blk.size())) != TDDE_OK) return s;
    }
    if (o->n_s > 0) {
      sum_poly(o->s_poly, o->n_s, blk);
      if ((s = up((T**)&op.s_blk, blk.data(), blk.size())) != TDDE_OK) return s;
    }
  }
  if (op.has_chan) {
    if ((s = up((T**)&op.h_chan, o->h_chan, (size_t)nang * bsz * 2)) != TDDE_OK) return s;
  } else {
    op.h_chan = nullptr;
  }
  // Group terms (at most kMaxGroup per group) whose angular sparsity patterns nearly coincide: a
  // group's pattern is the union of its terms' patterns (a term absent from an entry has value 0
  // there), and the apply stages the angular combinations of all terms of a group from one gather.
  // A term joins a group when the group's multiply-adds (union entries x terms) stay within 1.5x
  // of gathering the two apart: merging saves gathers and round trips at a bounded arithmetic cost.
  {
    std::vector<int> g_first{0}, g_term, g_rowptr, g_col;
    std::vector<long> g_voff;
    std::vector<double> g_val;
    std::vector<char> used(o->n_terms, 0);
    // sorted distinct columns of row j of term m
    auto term_row = [&](int m, int j) {
      const int32_t* rp = o->a_rowptr + (size_t)m * (nang + 1);
      std::vector<int> cols(o->a_col + o->a_off[m] + rp[j], o->a_col + o->a_off[m] + rp[j + 1]);
      std::sort(cols.begin(), cols.end());
      cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
      return cols;
    };
    auto row_union = [](const std::vector<int>& a, const std::vector<int>& b) {
      std::vector<int> u;
      std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(u));
      return u;
    };
    // A_m[j][col], duplicates summed
    auto term_val = [&](int m, int j, int col) {
      const int32_t* rp = o->a_rowptr + (size_t)m * (nang + 1);
      double v = 0.0;
      for (int p = rp[j]; p < rp[j + 1]; ++p)
        if (o->a_col[o->a_off[m] + p] == col) v += tval[o->a_off[m] + p];
      return v;
    };
    for (int m = 0; m < o->n_terms; ++m) {
      if (used[m]) continue;
      std::vector<int> grp{m};
      used[m] = 1;
      std::vector<std::vector<int>> pat(nang);
      size_t n_pat = 0;
      for (int j = 0; j < nang; ++j) { pat[j] = term_row(m, j); n_pat += pat[j].size(); }
      for (int m2 = m + 1; m2 < o->n_terms && (int)grp.size() < kMaxGroup; ++m2) {
        if (used[m2]) continue;
        std::vector<std::vector<int>> u(nang);
        size_t n_u = 0, n_m2 = 0;
        for (int j = 0; j < nang; ++j) {
          const std::vector<int> r2 = term_row(m2, j);
          n_m2 += r2.size();
          u[j] = row_union(pat[j], r2);
          n_u += u[j].size();
        }
        const size_t kg = grp.size();
        if (2 * n_u * (kg + 1) <= 3 * (n_pat * kg + n_m2)) {
          grp.push_back(m2);
          used[m2] = 1;
          pat.swap(u);
          n_pat = n_u;
        }
      }
      const int base = (int)g_col.size();
      g_voff.push_back((long)g_val.size());
      int acc = 0;
      for (int j = 0; j < nang; ++j) {
        g_rowptr.push_back(base + acc);
        for (int col : pat[j]) {
          g_col.push_back(col);
          for (int q : grp) g_val.push_back(term_val(q, j, col));
        }
        acc += (int)pat[j].size();
      }
      g_rowptr.push_back(base + acc);
      for (int q : grp) g_term.push_back(q);
      g_first.push_back((int)g_term.size());
    }
    op.n_groups = (int)g_first.size() - 1;
    if ((s = upload(c, (int**)&op.g_first, g_first.data(), g_first.size())) != TDDE_OK) return s;
    if ((s = upload(c, (int**)&op.g_term, g_term.data(), g_term.size())) != TDDE_OK) return s;
    if ((s = upload(c, (int**)&op.g_rowptr, g_rowptr.data(), g_rowptr.size())) != TDDE_OK) return s;
    if ((s = upload(c, (int**)&op.g_col, g_col.data(), g_col.size())) != TDDE_OK) return s;
    if ((s = upload(c, (long**)&op.g_voff, g_voff.data(), g_voff.size())) != TDDE_OK) return s;
    if ((s = up((T**)&op.g_val, g_val.data(), g_val.size())) != TDDE_OK) return s;
  }
  if ((s = up((T**)&op.t_r, o->n_terms ? o->r_band : nullptr, (size_t)o->n_terms * bsz)) != TDDE_OK) return s;
  if ((s = upload(c, (int**)&op.t_mask, mask.data(), mask.size())) != TDDE_OK) return s;
  if ((s = upload(c, (int**)&op.t_field, o->field, (size_t)o->n_terms)) != TDDE_OK) return s;
  if ((s = upload(c, (double2**)&op.t_coef, (const double2*)o->coef, (size_t)o->n_terms)) != TDDE_OK) return s;
  return TDDE_OK;
}

template <typename T> static tdde_status alloc_kvec(tdde_ctx* c, KVec<T>& V, KVec<T>& Vnp, size_t n) {
  tdde_status s;
  c2_t<T>** ptrs[] = {&V.x, &V.r, &V.rh, &V.p, &V.ph, &V.v, &V.s, &V.sh, &V.t};
  for (auto* p : ptrs)
    if ((s = dev_alloc(c, p, n)) != TDDE_OK) return s;
  Vnp = V;
  Vnp.ph = V.p;
  Vnp.sh = V.s;
  return TDDE_OK;
}

tdde_status tdde_assemble(tdde_ctx* c, const tdde_operator_desc* o) {
  if (!c || !o) return fail(c, TDDE_ERR_ARG, "null argument");
  if (c->assembled) return fail(c, TDDE_ERR_STATE, "operator already assembled");
  const int nr = c->d.nr, nang = c->d.nang, hb = c->d.half_band, nb = 2 * hb + 1;
  if (!o->kappa) return fail(c, TDDE_ERR_ARG, "kappa is required");
  if (o->n_h < 0 || o->n_h > 4 || (o->n_h > 0 && !o->h_poly)) return fail(c, TDDE_ERR_ARG, "n_h must be 0..4 with h_poly");
  if (o->n_s < 0 || o->n_s > 3 || (o->n_s > 0 && !o->s_poly)) return fail(c, TDDE_ERR_ARG, "n_s must be 0..3 with s_poly");
  if (o->n_terms < 0 || o->n_terms > kMaxTerms) return fail(c, TDDE_ERR_ARG, "n_terms must be 0..128");
  if (o->n_terms > 0 && (!o->a_rowptr || !o->a_off || !o->a_col || !o->a_val || !o->r_band || !o->kpow || !o->coef ||
                         !o->field))
    return fail(c, TDDE_ERR_ARG, "coupling arrays missing");
  // validate CSR and fold kappa exponents into the values
  std::vector<int> rowptr_abs((size_t)o->n_terms * (nang + 1));
  std::vector<double> tval;
  std::vector<int> mask(o->n_terms);
  const int64_t nnz = o->n_terms ? o->a_off[o->n_terms] : 0;
  if (nnz > INT32_MAX) return fail(c, TDDE_ERR_ARG, "too many coupling nonzeros");
  tval.resize(nnz);
  for (int m = 0; m < o->n_terms; ++m) {
    const int64_t off = o->a_off[m], off1 = o->a_off[m + 1];
    const int32_t* rp = o->a_rowptr + (size_t)m * (nang + 1);
    if (off < 0 || off1 < off || rp[0] != 0 || rp[nang] != off1 - off)
      return fail(c, TDDE_ERR_ARG, "term " + std::to_string(m) + ": inconsistent row pointers / offsets");
    if (o->field[m] < 0 || o->field[m] >= c->d.n_fields)
      return fail(c, TDDE_ERR_ARG, "term " + std::to_string(m) + ": field index out of range");
    const int ka = o->kpow[2 * m], kb = o->kpow[2 * m + 1];
    if (ka < 0 || ka > 3 || kb < 0 || kb > 3) return fail(c, TDDE_ERR_ARG, "kappa exponents must be 0..3");
    for (int j = 0; j <= nang; ++j) {
      if (j < nang && rp[j + 1] < rp[j]) return fail(c, TDDE_ERR_ARG, "row pointers not monotone");
      rowptr_abs[(size_t)m * (nang + 1) + j] = (int)(off + rp[j]);
    }
    for (int j = 0; j < nang; ++j)
      for (int p = rp[j]; p < rp[j + 1]; ++p) {
        const int jj = o->a_col[off + p];
        if (jj < 0 || jj >= nang) return fail(c, TDDE_ERR_ARG, "column index out of range");
        tval[off + p] = std::pow(o->kappa[j], ka) * o->a_val[off + p] * std::pow(o->kappa[jj], kb);
      }
    mask[m] = 0;
    for (int sel = 0; sel < 4; ++sel) {
      const double* rb = o->r_band + ((size_t)m * 4 + sel) * nb * nr;
      for (size_t k = 0; k < (size_t)nb * nr; ++k)
        if (rb[k] != 0.0) { mask[m] |= 1 << sel; break; }
    }
  }
  tdde_status s;
  if ((s = build_devop<double>(c, o, c->op64, tval, rowptr_abs, mask)) != TDDE_OK) return s;
  if ((s = build_devop<float>(c, o, c->op32, tval, rowptr_abs, mask)) != TDDE_OK) return s;
  // host copies for the preconditioner
  const size_t bsz = (size_t)4 * nb * nr;
  c->kappa.assign(o->kappa, o->kappa + nang);
  c->n_h = o->n_h;
  c->n_s = o->n_s;
  c->has_chan = o->h_chan != nullptr;
  if (o->n_h) c->h_poly.assign(o->h_poly, o->h_poly + o->n_h * bsz);
  if (o->n_s) c->s_poly.assign(o->s_poly, o->s_poly + o->n_s * bsz);
  if (o->h_chan) c->h_chan.assign(o->h_chan, o->h_chan + (size_t)nang * bsz * 2);
  // factor blocks: one per channel with its own complex band, else one per distinct kappa
  c->block_of.assign(nang, 0);
  if (c->has_chan) {
    for (int j = 0; j < nang; ++j) c->block_of[j] = j;
    c->nblk = nang;
  } else {
    std::map<double, int> seen;
    for (int j = 0; j < nang; ++j) {
      auto it = seen.find(o->kappa[j]);
      if (it == seen.end()) it = seen.emplace(o->kappa[j], (int)seen.size()).first;
      c->block_of[j] = it->second;
    }
    c->nblk = (int)seen.size();
  }
  // workspace
  const size_t n = (size_t)c->d.batch * c->E;
  if ((s = alloc_kvec<double>(c, c->v64, c->v64np, n)) != TDDE_OK) return s;
  if ((s = alloc_kvec<float>(c, c->v32, c->v32np, n)) != TDDE_OK) return s;
  if ((s = dev_alloc(c, &c->bvec, n)) != TDDE_OK) return s;
  if ((s = dev_alloc(c, &c->bvec2, n)) != TDDE_OK) return s;
  if ((s = dev_alloc(c, &c->xalt, n)) != TDDE_OK) return s;
  if ((s = dev_alloc(c, &c->r64, n)) != TDDE_OK) return s;
  if ((s = dev_alloc(c, &c->rhs32, n)) != TDDE_OK) return s;
  if ((s = dev_alloc(c, &c->fvals, (size_t)c->d.batch * c->d.n_fields)) != TDDE_OK) return s;
  if ((s = dev_alloc(c, &c->pulses, (size_t)c->d.batch * c->d.n_fields)) != TDDE_OK) return s;
  if ((s = dev_alloc(c, &c->n_steps_dev, (size_t)c->d.batch)) != TDDE_OK) return s;
  // persistent grids: as many work-groups as can be co-resident, per kernel variant
  int dev = 0, ncu = 0, max_wg = 0;
  HIP_TRY(c, hipGetDevice(&dev));
  HIP_TRY(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  for (int v = 0; v < 4; ++v) {
    int per_cu = 0;
    HIP_TRY(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_variant(v), kThreads, 0));
    if (per_cu <= 0) return fail(c, TDDE_ERR_HIP, "persistent kernel cannot be resident");
    c->var_occ[v] = per_cu;
    c->var_wg[v] = ncu * std::min(per_cu, kMaxWgPerCu);
    if (c->d.batch > c->var_wg[v]) return fail(c, TDDE_ERR_ARG, "batch larger than the co-resident work-group count");
    max_wg = std::max(max_wg, c->var_wg[v]);
  }
  c->ncu = ncu;
  c->n_wg = c->var_wg[0];
  c->G = c->n_wg / c->d.batch;
  if ((s = dev_alloc(c, &c->part, (size_t)max_wg * kSlots)) != TDDE_OK) return s;
  if ((s = dev_alloc(c, &c->bar, kBarWords)) != TDDE_OK) return s;
  c->n_counters = 64 * kCounterPerStep;
  if ((s = dev_alloc(c, &c->counters, (size_t)c->n_counters)) != TDDE_OK) return s;
  c->stats_cap = c->d.batch;
  if ((s = dev_alloc(c, &c->stats_dev, (size_t)c->stats_cap)) != TDDE_OK) return s;
  HIP_TRY(c, hipDeviceSynchronize());
  c->assembled = true;
  return TDDE_OK;
}

tdde_status tdde_debug_phase_marks(tdde_ctx* c, int32_t cap) {
  if (!c || cap < 0) return fail(c, TDDE_ERR_ARG, "bad argument");
  if (!c->assembled) return fail(c, TDDE_ERR_STATE, "assemble first");
  if (cap > c->n_marks) {
    tdde_status s = dev_alloc(c, &c->marks, (size_t)cap);
    if (s != TDDE_OK) return s;
  }
  if (cap == 0) c->marks = nullptr;
  c->n_marks = cap;
  return TDDE_OK;
}

tdde_status tdde_debug_read_marks(tdde_ctx* c, uint64_t* host, int32_t cap) {
  if (!c || !host || cap < 0) return fail(c, TDDE_ERR_ARG, "bad argument");
  if (!c->marks) return fail(c, TDDE_ERR_STATE, "enable phase marks first");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipMemcpy(host, c->marks, (size_t)std::min(cap, c->n_marks) * sizeof(uint64_t), hipMemcpyDeviceToHost));
  return TDDE_OK;
}

tdde_status tdde_set_graph(tdde_ctx* c, int32_t on) {
  if (!c) return fail(c, TDDE_ERR_ARG, "null context");
  c->use_graph = on != 0;
  return TDDE_OK;
}

tdde_status tdde_set_prec_segment(tdde_ctx* c, int32_t min_rows) {
  if (!c) return fail(c, TDDE_ERR_ARG, "null context");
  if (min_rows < 2 * c->d.half_band + 1 || min_rows > 4096)
    return fail(c, TDDE_ERR_ARG, "min_rows must be at least the factor band width (13) and at most 4096");
  c->seg_min = min_rows;
  return TDDE_OK;
}

// Work-groups per instance of the kernel-per-window solver's apply and vector kernels: two per CU
// over the batch, the apply kernels' occupancy, so the whole grid is resident at once and every XCD
// sweeps the channels of its radial tiles together (the neighbouring channels' tiles that the angular
// gathers read are then still in its L2; a grid of two rounds measured 3 % slower per step, its second
// half of work-groups starting only after the first had finished all of their tiles); a multiple of 8
// so that work-group g of every instance runs on XCD g % 8, and no more than the instance has tiles
// (rounded up to 8).
static int split_wg(const tdde_ctx* c) {
  const long tiles = (long)c->op64.nang * c->op64.n_itiles;
  long g = (2L * c->ncu / c->d.batch) / 8 * 8;
  g = std::max(8L, std::min(g, (tiles + 7) / 8 * 8));
  return (int)g;
}

tdde_status tdde_set_split(tdde_ctx* c, int32_t on) {
  if (!c) return fail(c, TDDE_ERR_ARG, "null context");
  if (!c->assembled) return fail(c, TDDE_ERR_STATE, "assemble first");
  if (on != 0 && on != 1) return fail(c, TDDE_ERR_ARG, "on must be 0 or 1");
  if (on && !c->sp_ctl) {
    const int G = split_wg(c);
    const size_t B = (size_t)c->d.batch;
    if ((double)B * G > 2.0e9) return fail(c, TDDE_ERR_ARG, "batch too large for the kernel-per-window grid");
    tdde_status s;
    if ((s = dev_alloc(c, &c->sp_ctl, B)) != TDDE_OK) return s;
    if ((s = dev_alloc(c, &c->sp_cnt, B * kSpCntLine)) != TDDE_OK) return s;
    if ((s = dev_alloc(c, &c->sp_part, B * G * kSpSlots)) != TDDE_OK) return s;
    HIP_TRY(c, hipHostMalloc(reinterpret_cast<void**>(&c->sp_flag), 2 * sizeof(int), hipHostMallocCoherent));
    c->sp_flag[0] = c->sp_flag[1] = -1;
    for (hipEvent_t& e : c->sp_ev) HIP_TRY(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->sp_G = G;
  }
  c->split = on != 0;
  return TDDE_OK;
}

tdde_status tdde_set_prec_storage(tdde_ctx* c, int32_t bits) {
  if (!c) return fail(c, TDDE_ERR_ARG, "null context");
  if (bits != 32 && bits != 64) return fail(c, TDDE_ERR_ARG, "bits must be 32 or 64");
  c->prec_f32 = bits == 32;
  return TDDE_OK;
}

tdde_status tdde_debug_split_timing(tdde_ctx* c, int32_t cap) {
  if (!c || cap < 0 || cap > (1 << 16)) return fail(c, TDDE_ERR_ARG, "cap must be 0..65536");
  while ((int)c->sp_tev.size() < 2 * cap) {
    hipEvent_t e = nullptr;
    HIP_TRY(c, hipEventCreate(&e));
    c->sp_tev.push_back(e);
  }
  c->sp_tcap = cap;
  c->sp_tn = 0;
  return TDDE_OK;
}

tdde_status tdde_debug_read_split_timing(tdde_ctx* c, float* ms, int32_t cap_host, int32_t* n) {
  if (!c || !n || (cap_host > 0 && !ms) || cap_host < 0) return fail(c, TDDE_ERR_ARG, "bad argument");
  const int k = std::min(c->sp_tn, cap_host);
  for (int i = 0; i < k; ++i) {
    HIP_TRY(c, hipEventSynchronize(c->sp_tev[2 * (size_t)i + 1]));
    HIP_TRY(c, hipEventElapsedTime(ms + i, c->sp_tev[2 * (size_t)i], c->sp_tev[2 * (size_t)i + 1]));
  }
  *n = k;
  c->sp_tn = 0;
  return TDDE_OK;
}

tdde_status tdde_debug_set_shadow(tdde_ctx* c, const void* shadow) {
  if (!c) return fail(c, TDDE_ERR_ARG, "null context");
  c->shadow = static_cast<const double2*>(shadow);
  return TDDE_OK;
}

tdde_status tdde_set_launch(tdde_ctx* c, int32_t wg_per_cu) {
  if (!c) return fail(c, TDDE_ERR_ARG, "null context");
  if (!c->assembled) return fail(c, TDDE_ERR_STATE, "assemble first");
  if (wg_per_cu < 0 || wg_per_cu > kMaxWgPerCu) return fail(c, TDDE_ERR_ARG, "wg_per_cu must be 0..4");
  const int k = wg_per_cu == 0 ? kMaxWgPerCu : wg_per_cu;
  int wg[4];
  for (int v = 0; v < 4; ++v) {
    wg[v] = c->ncu * std::min(c->var_occ[v], k);
    if (c->d.batch > wg[v]) return fail(c, TDDE_ERR_ARG, "batch larger than the requested work-group count");
  }
  // the partial-sum buffer was sized for the largest grid at assembly; grids only shrink here
  for (int v = 0; v < 4; ++v) c->var_wg[v] = wg[v];
  c->n_wg = c->var_wg[0];
  c->G = c->n_wg / c->d.batch;
  return TDDE_OK;
}

tdde_status tdde_launch_info(tdde_ctx* c, int32_t* n_wg, int32_t* per_inst) {
  if (!c || !n_wg || !per_inst) return fail(c, TDDE_ERR_ARG, "null argument");
  if (!c->assembled) return fail(c, TDDE_ERR_STATE, "assemble first");
  if (c->split) {
    *n_wg = c->sp_G * c->d.batch;
    *per_inst = c->sp_G;
  } else {
    *n_wg = c->n_wg;
    *per_inst = c->G;
  }
  return TDDE_OK;
}

// Chain work order: the channels of every factor block (channels of one distinct kappa share their
// LU factors) taken nc at a time into work items, blocks dealt to the 8 XCDs greedily by item count,
// and the list of XCD x placed at positions w = 8 i + x. Work-group w mod G (G a multiple of 8) runs on
// XCD w % 8, so the items of a block run side by side on one XCD and read its factor rows through that
// XCD's L2 instead of from memory once per XCD. Returns [n_items][nc] channels, -1 for none.
static std::vector<int> chain_order_of(const std::vector<int>& block_of, int nblk, int nc) {
  constexpr int kXcd = 8;
  std::vector<std::vector<int>> members(nblk);
  for (int j = 0; j < (int)block_of.size(); ++j) members[block_of[j]].push_back(j);
  std::vector<int> blocks(nblk);
  for (int b = 0; b < nblk; ++b) blocks[b] = b;
  std::stable_sort(blocks.begin(), blocks.end(),
                   [&](int a, int b) { return members[a].size() > members[b].size(); });
  std::vector<std::vector<std::vector<int>>> lists(kXcd);
  for (int b : blocks) {
    int best = 0;
    for (int x = 1; x < kXcd; ++x)
      if (lists[x].size() < lists[best].size()) best = x;
    const auto& mb = members[b];
    for (size_t i = 0; i < mb.size(); i += nc)
      lists[best].push_back(std::vector<int>(mb.begin() + i, mb.begin() + std::min(mb.size(), i + nc)));
  }
  size_t len = 0;
  for (auto& l : lists) len = std::max(len, l.size());
  std::vector<int> order(len * kXcd * nc, -1);
  for (int x = 0; x < kXcd; ++x)
    for (size_t i = 0; i < lists[x].size(); ++i)
      for (size_t k = 0; k < lists[x][i].size(); ++k) order[(i * kXcd + x) * nc + k] = lists[x][i][k];
  return order;
}

// Banded LU of M = S + i dt/2 H0 for one block, rows q = 2 i + s, plus segment coupling matrices.
static void factor_block(const tdde_ctx* c, int j, double dt, int m, int P, std::vector<cd>& LU, std::vector<cd>& TL,
                         std::vector<cd>& TU, std::vector<cd>& CL, std::vector<cd>& CU) {
  const int nr = c->d.nr, hb = c->d.half_band, n = 2 * nr, w = 2 * hb + 1, ws = 2 * w + 1;
  const double kap = c->kappa[j];
  std::vector<cd> A((size_t)n * ws, cd(0, 0));  // A[q][k + w] = M(q, q + k)
  for (int s = 0; s < 2; ++s)
    for (int s2 = 0; s2 < 2; ++s2)
      for (int d = -hb; d <= hb; ++d)
        for (int i = 0; i < nr; ++i) {
          const int i2 = i + d;
          if (i2 < 0 || i2 >= nr) continue;
          const int bi = band_index(hb, nr, s, s2, d, i);
          double sv = 0.0, hv = 0.0, hvi = 0.0, kn = 1.0;
          for (int k = 0; k < c->n_s; ++k, kn *= kap) sv += kn * c->s_poly[(size_t)k * 4 * (2 * hb + 1) * nr + bi];
          if (c->n_s == 0 && d == 0 && s == s2) sv = 1.0;
          kn = 1.0;
          for (int k = 0; k < c->n_h; ++k, kn *= kap) hv += kn * c->h_poly[(size_t)k * 4 * (2 * hb + 1) * nr + bi];
          if (c->has_chan) {
            const size_t ci = ((size_t)j * 4 * (2 * hb + 1) * nr + bi) * 2;
            hv += c->h_chan[ci];
            hvi += c->h_chan[ci + 1];
          }
          // M = S + i dt/2 (hv + i hvi)
          const cd val = cd(sv, 0.0) + cd(0.0, 0.5 * dt) * cd(hv, hvi);
          const int q = 2 * i + s, q2 = 2 * i2 + s2;
          A[(size_t)q * ws + (q2 - q) + w] += val;
        }
  for (int q = 0; q < n; ++q) {
    const cd piv = A[(size_t)q * ws + w];
    for (int r = q + 1; r <= std::min(q + w, n - 1); ++r) {
      cd& arq = A[(size_t)r * ws + (q - r) + w];
      if (arq == cd(0, 0)) continue;
      const cd l = arq / piv;
      arq = l;
      for (int cc = q + 1; cc <= std::min(q + w, n - 1); ++cc)
        A[(size_t)r * ws + (cc - r) + w] -= l * A[(size_t)q * ws + (cc - q) + w];
    }
  }
  auto Lq = [&](int q, int col) -> cd { return (col < 0 || q - col > w || col >= q) ? cd(0, 0) : A[(size_t)q * ws + (col - q) + w]; };
  auto Uq = [&](int q, int col) -> cd { return (col >= n || col - q > w || col <= q) ? cd(0, 0) : A[(size_t)q * ws + (col - q) + w]; };
  LU.assign((size_t)n * ws, cd(0, 0));
  for (int q = 0; q < n; ++q) {
    for (int k = 0; k < w; ++k) LU[(size_t)q * ws + k] = Lq(q, q - 1 - k);
    LU[(size_t)q * ws + w] = cd(1.0, 0.0) / A[(size_t)q * ws + w];
    for (int k = 0; k < w; ++k) LU[(size_t)q * ws + w + 1 + k] = Uq(q, q + 1 + k);
  }
  TL.assign((size_t)P * w * w, cd(0, 0));
  TU.assign((size_t)P * w * w, cd(0, 0));
  std::vector<cd> W;
  for (int p = 0; p < P; ++p) {
    const int o = p * m, len = std::min(m, n - o);
    if (p >= 1) {  // lower: W = L_pp^-1 C_p, C_p[r][c] = L(o + r, o - w + c)
      W.assign((size_t)len * w, cd(0, 0));
      for (int r = 0; r < len; ++r)
        for (int cc = 0; cc < w; ++cc) {
          cd v = Lq(o + r, o - w + cc);
          for (int k = 1; k <= w && r - k >= 0; ++k) v -= Lq(o + r, o + r - k) * W[(size_t)(r - k) * w + cc];
          W[(size_t)r * w + cc] = v;
        }
      for (int rr = 0; rr < w; ++rr)
        for (int cc = 0; cc < w; ++cc) TL[((size_t)p * w + rr) * w + cc] = W[(size_t)(len - w + rr) * w + cc];
    }
    if (p <= P - 2) {  // upper: W = U_pp^-1 D_p, D_p[r][c] = U(o + r, o + len + c)
      W.assign((size_t)len * w, cd(0, 0));
      const int o2 = o + len;
      for (int r = len - 1; r >= 0; --r)
        for (int cc = 0; cc < w; ++cc) {
          cd v = Uq(o + r, o2 + cc);
          for (int k = 1; k <= w && r + k < len; ++k) v -= Uq(o + r, o + r + k) * W[(size_t)(r + k) * w + cc];
          W[(size_t)r * w + cc] = v * LU[(size_t)(o + r) * ws + w];
        }
      for (int rr = 0; rr < w; ++rr)
        for (int cc = 0; cc < w; ++cc) TU[((size_t)p * w + rr) * w + cc] = W[(size_t)rr * w + cc];
    }
  }
  // Group products for the two-level boundary propagation (segments in groups of kSegGroup):
  // lower, p in group G >= 1 with first segment f = G * kSegGroup:
  //   CL_p = (-T_p)(-T_{p-1}) ... (-T_f), so that t_p = t^loc_p + CL_p u_{G-1}
  // (t^loc: the group's recurrence started from a zero window, u_{G-1}: true tail of the last
  // segment of group G-1); upper likewise from the top segment of every group but the last.
  auto mul_neg = [&](const cd* A, const cd* B, cd* C) {  // C = -A B (w x w)
    for (int r = 0; r < w; ++r)
      for (int cc = 0; cc < w; ++cc) {
        cd acc(0, 0);
        for (int k = 0; k < w; ++k) acc += A[r * w + k] * B[k * w + cc];
        C[r * w + cc] = -acc;
      }
  };
  std::vector<cd> CLp((size_t)P * w * w, cd(0, 0)), CUp((size_t)P * w * w, cd(0, 0));  // [p][w][w]
  const int last_group = (P - 1) / kSegGroup;
  for (int p = 0; p < P; ++p) {
    const int G = p / kSegGroup;
    if (G == 0) continue;
    cd* dst = CLp.data() + (size_t)p * w * w;
    const cd* T = TL.data() + (size_t)p * w * w;
    if (p == G * kSegGroup) {
      for (int k = 0; k < w * w; ++k) dst[k] = -T[k];
    } else {
      mul_neg(T, CLp.data() + (size_t)(p - 1) * w * w, dst);
    }
  }
  for (int p = P - 1; p >= 0; --p) {
    const int G = p / kSegGroup;
    if (G == last_group) continue;
    cd* dst = CUp.data() + (size_t)p * w * w;
    const cd* T = TU.data() + (size_t)p * w * w;
    if (p == G * kSegGroup + kSegGroup - 1) {
      for (int k = 0; k < w * w; ++k) dst[k] = -T[k];
    } else {
      mul_neg(T, CUp.data() + (size_t)(p + 1) * w * w, dst);
    }
  }
  // device layout [w][w][p]: threads of consecutive segments read consecutive entries
  CL.assign((size_t)P * w * w, cd(0, 0));
  CU.assign((size_t)P * w * w, cd(0, 0));
  for (int p = 0; p < P; ++p)
    for (int k = 0; k < w * w; ++k) {
      CL[(size_t)k * P + p] = CLp[(size_t)p * w * w + k];
      CU[(size_t)k * P + p] = CUp[(size_t)p * w * w + k];
    }
}

tdde_status tdde_set_dt(tdde_ctx* c, double dt) {
  if (!c) return TDDE_ERR_ARG;
  if (!c->assembled) return fail(c, TDDE_ERR_STATE, "assemble first");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, TDDE_ERR_ARG, "dt must be positive and finite");
  c->dt = dt;
  c->dt_set = true;
  const int nr = c->d.nr, hb = c->d.half_band, n = 2 * nr, w = 2 * hb + 1, ws = 2 * w + 1;
  if (w != kPrecW) return TDDE_OK;  // preconditioner available for half_band 6 only (checked at solve)
  if (n < w) return TDDE_OK;
  // Segments of at least 24 rows: two thirds of the segment-boundary matrices (T, C) of 16-row
  // segments, so more of the factors stay resident in the Infinity Cache beside the solver's vectors
  // between two solves (hydrogen: 147 MB instead of 186 MB). Measured on the hydrogen step, 24 rows
  // beat 16, 32, 40 and 48 (longer segments lengthen each thread's substitution chain).
  const int m = std::max({w, c->seg_min, (n + kMaxSeg - 1) / kMaxSeg});
  const int P = (n + m - 1) / m;
  std::vector<cd> LU, TL, TU, CL, CU;
  const size_t tsz = (size_t)P * w * w;
  const size_t lsz = (size_t)m * ws * P;  // per block: [m][ws][P], segment index fastest
  std::vector<cd> allLU(c->nblk * lsz, cd(0, 0)), allTL(c->nblk * tsz), allTU(c->nblk * tsz), allCL(c->nblk * tsz),
      allCU(c->nblk * tsz);
  std::vector<int> rep(c->nblk, -1);
  for (int j = 0; j < c->d.nang; ++j)
    if (rep[c->block_of[j]] < 0) rep[c->block_of[j]] = j;
  for (int bk = 0; bk < c->nblk; ++bk) {
    factor_block(c, rep[bk], dt, m, P, LU, TL, TU, CL, CU);
    cd* lu = allLU.data() + bk * lsz;
    for (int q = 0; q < n; ++q) {
      const int sg = q / m, t = q - sg * m;
      for (int k = 0; k < ws; ++k) lu[((size_t)t * ws + k) * P + sg] = LU[(size_t)q * ws + k];
    }
    // T_p stored transposed: [p][c][r]
    for (int sg = 0; sg < P; ++sg)
      for (int r = 0; r < w; ++r)
        for (int cc = 0; cc < w; ++cc) {
          allTL[bk * tsz + ((size_t)sg * w + cc) * w + r] = TL[((size_t)sg * w + r) * w + cc];
          allTU[bk * tsz + ((size_t)sg * w + cc) * w + r] = TU[((size_t)sg * w + r) * w + cc];
        }
    std::copy(CL.begin(), CL.end(), allCL.begin() + bk * tsz);
    std::copy(CU.begin(), CU.end(), allCU.begin() + bk * tsz);
  }
  tdde_status s;
  if (!c->prec_alloc || allLU.size() > c->cap_lu || allTL.size() > c->cap_t) {
    // first factorisation, or a segment length whose factors need more room (earlier buffers stay
    // allocated until tdde_destroy)
    c->cap_lu = allLU.size();
    c->cap_t = allTL.size();
    if ((s = dev_alloc(c, (double2**)&c->pc64.LU, allLU.size())) != TDDE_OK) return s;
    if ((s = dev_alloc(c, (double2**)&c->pc64.TL, allTL.size())) != TDDE_OK) return s;
    if ((s = dev_alloc(c, (double2**)&c->pc64.TU, allTU.size())) != TDDE_OK) return s;
    if ((s = dev_alloc(c, (double2**)&c->pc64.CL, allCL.size())) != TDDE_OK) return s;
    if ((s = dev_alloc(c, (double2**)&c->pc64.CU, allCU.size())) != TDDE_OK) return s;
    if ((s = dev_alloc(c, (float2**)&c->pc32.LU, allLU.size())) != TDDE_OK) return s;
    if ((s = dev_alloc(c, (float2**)&c->pc32.TL, allTL.size())) != TDDE_OK) return s;
    if ((s = dev_alloc(c, (float2**)&c->pc32.TU, allTU.size())) != TDDE_OK) return s;
    if ((s = dev_alloc(c, (float2**)&c->pc32.CL, allCL.size())) != TDDE_OK) return s;
    if ((s = dev_alloc(c, (float2**)&c->pc32.CU, allCU.size())) != TDDE_OK) return s;
  }
  if (!c->prec_alloc) {
    if ((s = upload(c, (int**)&c->pc64.block_of, c->block_of.data(), c->block_of.size())) != TDDE_OK) return s;
    c->pc32.block_of = c->pc64.block_of;
    // chain order for every channel count per work-group (nc <= 8: at most nang + 8 nblk items)
    c->order_cap = (c->d.nang + 8 * (size_t)c->nblk) * kMaxChainNc;
    if ((s = dev_alloc(c, (int**)&c->pc64.chain_order, c->order_cap)) != TDDE_OK) return s;
    c->pc32.chain_order = c->pc64.chain_order;
    c->prec_alloc = true;
  }
  c->pc64.n = c->pc32.n = n;
  c->pc64.m = c->pc32.m = m;
  c->pc64.P = c->pc32.P = P;
  {
    // channels per chain work-group: as many as fit 256 lanes at P segments each (a power of two, so
    // that every channel's segment groups fit its kMaxSegGroups / nc slots)
    int nc = 1;
    while (nc < kMaxChainNc && 2 * nc * P <= kMaxSeg) nc *= 2;
    const std::vector<int> order = chain_order_of(c->block_of, c->nblk, nc);
    if (order.size() > c->order_cap) return fail(c, TDDE_ERR_HIP, "chain order larger than its buffer");
    HIP_TRY(c, hipMemcpy((void*)c->pc64.chain_order, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice));
    c->pc64.nc = c->pc32.nc = nc;
    c->pc64.n_items = c->pc32.n_items = (int)(order.size() / nc);
  }
  auto tof = [](const std::vector<cd>& v) {
    std::vector<float> f(2 * v.size());
    for (size_t i = 0; i < v.size(); ++i) { f[2 * i] = (float)v[i].real(); f[2 * i + 1] = (float)v[i].imag(); }
    return f;
  };
  const std::vector<cd>* host[] = {&allLU, &allTL, &allTU, &allCL, &allCU};
  const void* dev64[] = {c->pc64.LU, c->pc64.TL, c->pc64.TU, c->pc64.CL, c->pc64.CU};
  const void* dev32[] = {c->pc32.LU, c->pc32.TL, c->pc32.TU, c->pc32.CL, c->pc32.CU};
  for (int k = 0; k < 5; ++k) {
    HIP_TRY(c, hipMemcpy((void*)dev64[k], host[k]->data(), host[k]->size() * sizeof(cd), hipMemcpyHostToDevice));
    const std::vector<float> f = tof(*host[k]);
    HIP_TRY(c, hipMemcpy((void*)dev32[k], f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
  }
  return TDDE_OK;
}

tdde_status tdde_set_pulses(tdde_ctx* c, const tdde_pulse* p) {
  if (!c || !p) return fail(c, TDDE_ERR_ARG, "null argument");
  if (!c->assembled) return fail(c, TDDE_ERR_STATE, "assemble first");
  const size_t n = (size_t)c->d.batch * c->d.n_fields;
  std::vector<PulseDev> h(n);
  for (size_t i = 0; i < n; ++i) {
    if (!(p[i].T > 0.0)) return fail(c, TDDE_ERR_ARG, "pulse duration must be positive");
    h[i] = PulseDev{p[i].amp, p[i].T, p[i].omega, p[i].phase, p[i].envelope, 0};
  }
  HIP_TRY(c, hipMemcpyAsync(c->pulses, h.data(), n * sizeof(PulseDev), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->pulses_set = true;
  c->use_table = false;
  return TDDE_OK;
}

tdde_status tdde_set_field_table(tdde_ctx* c, const double* f, int32_t n_rows) {
  if (!c || !f) return fail(c, TDDE_ERR_ARG, "null argument");
  if (!c->assembled) return fail(c, TDDE_ERR_STATE, "assemble first");
  if (n_rows < 1) return fail(c, TDDE_ERR_ARG, "n_rows must be positive");
  const size_t n = (size_t)c->d.batch * n_rows * c->d.n_fields;
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(f[i])) return fail(c, TDDE_ERR_ARG, "field table values must be finite");
  if (n > c->ftab_cap) {
    tdde_status s = dev_alloc(c, &c->ftab, n);  // the smaller table stays allocated until destroy
    if (s != TDDE_OK) return s;
    c->ftab_cap = n;
  }
  HIP_TRY(c, hipMemcpyAsync(c->ftab, f, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->ftab_rows = n_rows;
  c->use_table = true;
  return TDDE_OK;
}

__global__ void eval_pulses_kernel(const PulseDev* pulses, int B, int nf, double t0, int step0, int n, double dt,
                                   double* out) {
  const int total = B * n * nf;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int m = i % nf, k = (i / nf) % n, b = i / (nf * n);
    out[i] = pulse_eval(pulses[(size_t)b * nf + m], mid_time(t0, step0 + k, dt));
  }
}

tdde_status tdde_eval_pulses(tdde_ctx* c, double t0, int32_t step0, int32_t n, double* f) {
  if (!c || !f) return fail(c, TDDE_ERR_ARG, "null argument");
  if (!c->assembled || !c->dt_set || !c->pulses_set) return fail(c, TDDE_ERR_STATE, "assemble, set_dt, set_pulses first");
  if (n < 1) return fail(c, TDDE_ERR_ARG, "n must be positive");
  const size_t total = (size_t)c->d.batch * n * c->d.n_fields;
  // the values go through the right-hand-side workspace (2 * batch * E doubles)
  if (total > (size_t)2 * c->d.batch * c->E) return fail(c, TDDE_ERR_ARG, "too many values for the workspace");
  double* out = reinterpret_cast<double*>(c->bvec);
  hipLaunchKernelGGL(eval_pulses_kernel, dim3((unsigned)std::min<size_t>((total + 255) / 256, 4096)), dim3(256), 0,
                     c->stream, c->pulses, c->d.batch, c->d.n_fields, t0, step0, n, c->dt, out);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipMemcpyAsync(f, out, total * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return TDDE_OK;
}

tdde_status tdde_set_field(tdde_ctx* c, const double* f) {
  if (!c || !f) return fail(c, TDDE_ERR_ARG, "null argument");
  if (!c->assembled) return fail(c, TDDE_ERR_STATE, "assemble first");
  HIP_TRY(c, hipMemcpyAsync(c->fvals, f, (size_t)c->d.batch * c->d.n_fields * sizeof(double), hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->field_set = true;
  return TDDE_OK;
}

template <typename T>
static tdde_status launch_apply(tdde_ctx* c, const DevOp<T>& op, tdde_c128 as, tdde_c128 ah, const void* x, void* y) {
  if (!c || !x || !y) return fail(c, TDDE_ERR_ARG, "null argument");
  if (!c->assembled || !c->field_set) return fail(c, TDDE_ERR_STATE, "assemble and set_field first");
  if (x == y) return fail(c, TDDE_ERR_ARG, "x and y must differ");
  const long n_tiles = (long)op.nang * op.n_itiles;
  const long n_wg = (n_tiles + 7) / 8 * 8 * c->d.batch;  // tile_coords order, every instance (apply_kernel)
  if (n_wg > INT32_MAX) return fail(c, TDDE_ERR_ARG, "too many tiles for one launch");
  hipLaunchKernelGGL(apply_kernel<T>, dim3((unsigned)n_wg), dim3(kThreads), 0, c->stream, op, (const c2_t<T>*)x,
                     (c2_t<T>*)y, make_double2(as.re, as.im), make_double2(ah.re, ah.im), (const double*)c->fvals,
                     c->d.n_fields, c->E, c->d.batch);
  HIP_TRY(c, hipGetLastError());
  return TDDE_OK;
}

tdde_status tdde_apply(tdde_ctx* c, tdde_c128 as, tdde_c128 ah, const void* x, void* y) {
  return c ? launch_apply<double>(c, c->op64, as, ah, x, y) : TDDE_ERR_ARG;
}
tdde_status tdde_apply_c64(tdde_ctx* c, tdde_c128 as, tdde_c128 ah, const void* x, void* y) {
  return c ? launch_apply<float>(c, c->op32, as, ah, x, y) : TDDE_ERR_ARG;
}

tdde_status tdde_precond_apply(tdde_ctx* c, const void* v, void* z) {
  if (!c || !v || !z) return fail(c, TDDE_ERR_ARG, "null argument");
  if (!c->dt_set || !c->prec_alloc) return fail(c, TDDE_ERR_STATE, "set_dt first (half_band 6 only)");
  if (v == z) return fail(c, TDDE_ERR_ARG, "input and output must differ");
  hipLaunchKernelGGL(precond_kernel<double>, dim3(c->pc64.n_items, c->d.batch), dim3(kThreads), 0, c->stream, c->pc64, c->d.nr,
                     (const double2*)v, (double2*)z, c->E);
  HIP_TRY(c, hipGetLastError());
  return TDDE_OK;
}

static tdde_status check_opts(tdde_ctx* c, const tdde_solve_opts* o) {
  if (!o) return fail(c, TDDE_ERR_ARG, "null options");
  if (!(o->tol > 0.0) || o->max_iter <= 0) return fail(c, TDDE_ERR_ARG, "tol > 0 and max_iter > 0 required");
  if (o->guess < 0 || o->guess > 2) return fail(c, TDDE_ERR_ARG, "unknown guess mode");
  if (o->precision != TDDE_PREC_FP64 && o->precision != TDDE_PREC_MIXED) return fail(c, TDDE_ERR_ARG, "precision");
  if (o->precision == TDDE_PREC_MIXED && (!(o->inner_tol > 0.0) || o->max_outer <= 0 || o->max_outer > 60))
    return fail(c, TDDE_ERR_ARG, "mixed precision needs inner_tol > 0 and 1 <= max_outer <= 60");
  if (o->precond && !c->prec_alloc) return fail(c, TDDE_ERR_STATE, "preconditioner needs set_dt and half_band 6");
  return TDDE_OK;
}

// Graph mode: capture [fill counters, fill barrier words, cooperative solver launch] on the
// context's stream once per (variant, grid), then replay it with this chunk's arguments set on the
// captured kernel nodes. Capture needs a stream other than the legacy default stream; a HIP error
// on the way (a runtime that does not capture cooperative launches) is returned as TDDE_ERR_HIP
// with its message.
static tdde_status run_graph(tdde_ctx* c, SolveArgs& a, int v, int n_chunk) {
  auto& cp = c->cap;
  const int n_cnt = 64 * kCounterPerStep;  // the whole counter array (independent of n_chunk)
  void* args[] = {&a};
  if (cp.v != v || cp.n_wg != c->n_wg) {
    if (cp.exec) { (void)hipGraphExecDestroy(cp.exec); cp.exec = nullptr; }
    if (cp.graph) { (void)hipGraphDestroy(cp.graph); cp.graph = nullptr; }
    cp.v = -1;
    HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipLaunchKernelGGL(zero_words, dim3(64), dim3(256), 0, c->stream, reinterpret_cast<unsigned*>(c->counters), n_cnt);
    hipLaunchKernelGGL(zero_words, dim3(8), dim3(256), 0, c->stream, c->bar, kBarWords);
    const hipError_t el = hipLaunchCooperativeKernel(persistent_variant(v), dim3(c->n_wg), dim3(kThreads), args, 0,
                                                     c->stream);
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(c->stream, &g);
    if (el != hipSuccess || ee != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(c, TDDE_ERR_HIP, std::string("graph capture of the cooperative launch: launch ") +
                                       hipGetErrorString(el) + ", end capture " + hipGetErrorString(ee));
    }
    cp.graph = g;
    size_t nn = 0;
    HIP_TRY(c, hipGraphGetNodes(g, nullptr, &nn));
    std::vector<hipGraphNode_t> nodes(nn);
    HIP_TRY(c, hipGraphGetNodes(g, nodes.data(), &nn));
    cp.solver = cp.zero_cnt = nullptr;
    for (hipGraphNode_t nd : nodes) {
      hipGraphNodeType ty;
      HIP_TRY(c, hipGraphNodeGetType(nd, &ty));
      if (ty != hipGraphNodeTypeKernel) continue;
      hipKernelNodeParams kp{};
      HIP_TRY(c, hipGraphKernelNodeGetParams(nd, &kp));
      if (kp.func == persistent_variant(v)) cp.solver = nd;
    }
    if (!cp.solver) return fail(c, TDDE_ERR_HIP, "graph capture: the solver kernel node was not recorded");
    HIP_TRY(c, hipGraphInstantiate(&cp.exec, g, nullptr, nullptr, 0));
    cp.v = v;
    cp.n_wg = c->n_wg;
  } else {
    hipKernelNodeParams kp{};
    HIP_TRY(c, hipGraphKernelNodeGetParams(cp.solver, &kp));
    kp.kernelParams = args;
    HIP_TRY(c, hipGraphExecKernelNodeSetParams(cp.exec, cp.solver, &kp));
  }
  HIP_TRY(c, hipGraphLaunch(cp.exec, c->stream));
  (void)n_chunk;
  return TDDE_OK;
}

static tdde_status run_persistent(tdde_ctx* c, SolveArgs& a, int n_chunk) {
  if (n_chunk > 64) return fail(c, TDDE_ERR_ARG, "at most 64 steps per launch");
  const int v = 2 * (a.mixed ? 1 : 0) + (a.use_prec ? 1 : 0);
  // work-groups per instance: a multiple of 8 keeps a tile of every instance on one XCD
  int G = c->var_wg[v] / c->d.batch;
  if (G >= 8) G -= G % 8;
  c->n_wg = c->var_wg[v];
  c->G = G;
  a.n_wg = c->n_wg;
  a.G = G;
  a.marks = c->marks;
  a.n_marks = c->n_marks;
  if (c->use_graph && a.counters == c->counters && a.bar == c->bar && !c->marks) return run_graph(c, a, v, n_chunk);
  // barrier words and per-step counters start at zero (a fill kernel, so the call can be captured)
  hipLaunchKernelGGL(zero_words, dim3(64), dim3(256), 0, c->stream, reinterpret_cast<unsigned*>(a.counters),
                     n_chunk * kCounterPerStep);
  hipLaunchKernelGGL(zero_words, dim3(8), dim3(256), 0, c->stream, a.bar, kBarWords);
  if (c->marks)
    hipLaunchKernelGGL(zero_words, dim3(16), dim3(256), 0, c->stream, reinterpret_cast<unsigned*>(c->marks),
                       2 * c->n_marks);
  HIP_TRY(c, hipGetLastError());
  void* args[] = {&a};
  HIP_TRY(c, hipLaunchCooperativeKernel(persistent_variant(v), dim3(c->n_wg), dim3(kThreads), args, 0, c->stream));
  return TDDE_OK;
}

static SolveArgs base_args(tdde_ctx* c, const tdde_solve_opts* o) {
  SolveArgs a{};
  a.op64 = c->op64;
  a.op32 = c->op32;
  a.pc64 = c->pc64;
  a.pc32 = c->pc32;
  a.use_prec = o->precond ? 1 : 0;
  a.v64 = a.use_prec ? c->v64 : c->v64np;
  a.v32 = a.use_prec ? c->v32 : c->v32np;
  a.bvec = c->bvec;
  a.bvec2 = c->bvec2;
  a.xalt = c->xalt;
  a.r64 = c->r64;
  a.rhs32 = c->rhs32;
  a.B = c->d.batch;
  a.E = c->E;
  a.guess = o->guess;
  a.mixed = o->precision == TDDE_PREC_MIXED;
  a.max_iter = o->max_iter;
  a.max_outer = o->max_outer;
  a.tol = o->tol;
  a.inner_tol = o->inner_tol;
  a.dt = c->dt;
  a.n_fields = c->d.n_fields;
  a.pulses = c->pulses;
  a.ftab = c->use_table ? c->ftab : nullptr;
  a.ftab_rows = c->ftab_rows;
  a.fvals = c->fvals;
  a.part = c->part;
  a.bar = c->bar;
  a.counters = c->counters;
  a.stats = c->stats_dev;
  a.shadow = c->shadow;
  a.n_chunk = 1;
  return a;
}

static_assert(sizeof(StatsDev) == sizeof(tdde_solve_stats) && offsetof(StatsDev, rel_res) ==
                  offsetof(tdde_solve_stats, rel_res) && offsetof(StatsDev, true_rel_res) ==
                  offsetof(tdde_solve_stats, true_rel_res),
              "device statistics must match the ABI struct");

// Copy the statistics of a single-step launch to the host (synchronises the stream); bar: the
// launch's grid-barrier words (time-out flag), null for the kernel-per-window solver.
static tdde_status collect_stats(tdde_ctx* c, tdde_solve_stats* out, const StatsDev* stats_dev, const unsigned* bar) {
  HIP_TRY(c, hipMemcpyAsync(out, stats_dev, (size_t)c->d.batch * sizeof(StatsDev), hipMemcpyDeviceToHost, c->stream));
  unsigned err_word = 0;
  if (bar) HIP_TRY(c, hipMemcpyAsync(&err_word, bar + kBarErr, sizeof(err_word), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (err_word != 0) return fail(c, TDDE_ERR_HIP, "grid barrier timed out (work-groups not co-resident)");
  tdde_status worst = TDDE_OK;
  for (int b = 0; b < c->d.batch; ++b) {
    if (out[b].status == TDDE_NONFINITE) worst = TDDE_NONFINITE;
    else if (out[b].status == TDDE_BREAKDOWN && worst != TDDE_NONFINITE) worst = TDDE_BREAKDOWN;
    else if (out[b].status != 0 && worst == TDDE_OK) worst = TDDE_NOT_CONVERGED;
  }
  return worst;
}
static tdde_status collect_stats(tdde_ctx* c, tdde_solve_stats* out) {
  return collect_stats(c, out, c->stats_dev, c->bar);
}

static tdde_status check_solve(tdde_ctx* c, const void* b, const void* x, const tdde_solve_opts* o) {
  if (!c || !b || !x) return fail(c, TDDE_ERR_ARG, "null argument");
  if (!c->assembled || !c->dt_set || !c->field_set) return fail(c, TDDE_ERR_STATE, "assemble, set_dt, set_field first");
  tdde_status s = check_opts(c, o);
  if (s != TDDE_OK) return s;
  if (o->guess == TDDE_GUESS_PREV) return fail(c, TDDE_ERR_ARG, "solve takes a ZERO or GIVEN guess");
  return TDDE_OK;
}

tdde_status tdde_solve(tdde_ctx* c, const void* b, void* x, const tdde_solve_opts* o, tdde_solve_stats* stats) {
  tdde_status s = check_solve(c, b, x, o);
  if (s != TDDE_OK) return s;
  SolveArgs a = base_args(c, o);
  a.mode = MODE_SOLVE;
  a.b_in = (const double2*)b;
  a.x_io = (double2*)x;
  if ((s = run_persistent(c, a, 1)) != TDDE_OK) return s;
  if (!stats) return TDDE_OK;
  return collect_stats(c, stats);
}

// Layout of the static scratch for one solve: 10 vectors of batch * E complex128 (iterate, r, r^, p,
// p^, v, s, s^, t, right-hand side), the reduction partials, the grid-barrier words, one step's
// counters and the statistics; every piece starts on a 256-byte boundary.
struct StaticLayout {
  size_t vec, part, bar, counters, stats, total;
};
static StaticLayout static_layout(const tdde_ctx* c) {
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  StaticLayout L{};
  const size_t n = (size_t)c->d.batch * c->E;
  L.vec = up(n * sizeof(double2));
  size_t off = 10 * L.vec;
  L.part = off;
  off += up((size_t)c->ncu * kMaxWgPerCu * kSlots * sizeof(double2));
  L.bar = off;
  off += up(kBarWords * sizeof(unsigned));
  L.counters = off;
  off += up(kCounterPerStep * sizeof(int));
  L.stats = off;
  off += up((size_t)c->d.batch * sizeof(StatsDev));
  L.total = off;
  return L;
}

tdde_status tdde_solve_static(tdde_ctx* c, const void* b, void* x, const tdde_solve_opts* o,
                              tdde_solve_stats* stats) {
  tdde_status s = check_solve(c, b, x, o);
  if (s != TDDE_OK) return s;
  if (o->precision != TDDE_PREC_FP64) return fail(c, TDDE_ERR_ARG, "tdde_solve_static runs the FP64 solver only");
  const StaticLayout L = static_layout(c);
  if (L.total > (size_t)TDDE_STATIC_SCRATCH_BYTES)
    return fail(c, TDDE_ERR_ARG, "tdde_solve_static: the solve needs " + std::to_string(L.total) +
                                     " bytes of scratch, more than the static array's " +
                                     std::to_string((long long)TDDE_STATIC_SCRATCH_BYTES) +
                                     " (batch * nang * 2 * nr too large)");
  int dev = 0;
  HIP_TRY(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(c, TDDE_ERR_HIP, "device index out of range");
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[dev])
      return fail(c, TDDE_ERR_STATE, "static scratch not resolved on this device (create the context with it current)");
    if (g_scratch_err[dev] != hipSuccess)
      return fail(c, TDDE_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(g_scratch_err[dev]));
    base = static_cast<unsigned char*>(g_scratch_dev[dev]);
  }
  SolveArgs a = base_args(c, o);
  double2* vec[10];
  for (int k = 0; k < 10; ++k) vec[k] = reinterpret_cast<double2*>(base + k * L.vec);
  KVec<double> V{vec[0], vec[1], vec[2], vec[3], vec[4], vec[5], vec[6], vec[7], vec[8]};
  if (!a.use_prec) { V.ph = V.p; V.sh = V.s; }
  a.v64 = V;
  a.v32 = KVec<float>{};
  a.bvec = vec[9];
  a.bvec2 = nullptr;  // single solve: no next step's right-hand side
  a.xalt = nullptr;   // single solve: no second iterate buffer
  a.r64 = nullptr;
  a.rhs32 = nullptr;
  a.part = reinterpret_cast<double2*>(base + L.part);
  a.bar = reinterpret_cast<unsigned*>(base + L.bar);
  a.counters = reinterpret_cast<int*>(base + L.counters);
  a.stats = reinterpret_cast<StatsDev*>(base + L.stats);
  a.mode = MODE_SOLVE;
  a.b_in = (const double2*)b;
  a.x_io = (double2*)x;
  if ((s = run_persistent(c, a, 1)) != TDDE_OK) return s;
  if (!stats) return TDDE_OK;
  return collect_stats(c, stats, a.stats, a.bar);
}

// Time steps by the kernel-per-window solver: blocks of kernels (one BiCGSTAB iteration of every
// unfinished instance each) are enqueued until the count of unfinished instances, read one block
// behind from host memory, reaches zero. Returns when every instance has finished its steps of the
// call (the stream then holds at most one block of kernels that find nothing to do).
static tdde_status run_split(tdde_ctx* c, const SolveArgs& a) {
  SplitArgs s{};
  s.op = c->op64;
  s.pc = c->pc64;
  s.pc32 = c->pc32;
  s.prec32 = c->prec_f32 ? 1 : 0;
  const KVec<double>& V = a.v64;
  s.x = a.psi;
  s.r = V.r;
  s.rh = V.rh;
  s.p = V.p;
  s.ph = V.ph;
  s.v = V.v;
  s.s = V.s;
  s.sh = V.sh;
  s.t = V.t;
  s.bvec[0] = c->bvec;
  s.bvec[1] = c->bvec2;
  s.part = c->sp_part;
  s.ctl = c->sp_ctl;
  s.cnt = c->sp_cnt;
  s.stats = a.stats;
  s.n_steps = a.n_steps;
  s.pulses = a.pulses;
  s.ftab = a.ftab;
  s.ftab_rows = a.ftab_rows;
  s.n_fields = a.n_fields;
  s.host_flag = c->sp_flag;
  s.B = c->d.batch;
  s.E = c->E;
  s.G = c->sp_G;
  s.step0 = a.step0;
  s.n_chunk = a.n_chunk;
  s.max_iter = a.max_iter;
  s.use_prec = a.use_prec;
  s.tol = a.tol;
  s.dt = a.dt;
  s.t0 = a.t0;
  // a step takes at most max_iter iterations, 21 restarts and one extra residual check, each at
  // least one block
  const long max_blocks = (long)a.n_chunk * ((long)a.max_iter + 24) + 4;
  for (long m = 0;; ++m) {
    const hipEvent_t* ev = nullptr;
    if (c->sp_tn < c->sp_tcap) ev = &c->sp_tev[2 * (size_t)c->sp_tn++];
    HIP_TRY(c, split_launch_block(s, c->stream, (int)(m & 1), m == 0, ev));
    HIP_TRY(c, hipEventRecord(c->sp_ev[m & 1], c->stream));
    if (m == 0) continue;
    HIP_TRY(c, hipEventSynchronize(c->sp_ev[(m - 1) & 1]));
    const int left = __atomic_load_n(c->sp_flag + ((m - 1) & 1), __ATOMIC_ACQUIRE);
    if (left == 0) break;
    if (m >= max_blocks) return fail(c, TDDE_ERR_HIP, "kernel-per-window solver did not finish its steps");
  }
  return TDDE_OK;
}

static bool split_serves(const tdde_ctx* c, const tdde_solve_opts* o) {
  return c->split && o->guess == TDDE_GUESS_PREV && o->precision == TDDE_PREC_FP64;
}

tdde_status tdde_step(tdde_ctx* c, void* psi, double t, const void* guess, const tdde_solve_opts* o,
                      tdde_solve_stats* stats) {
  if (!c || !psi) return fail(c, TDDE_ERR_ARG, "null argument");
  if (!c->assembled || !c->dt_set || !(c->pulses_set || c->use_table))
    return fail(c, TDDE_ERR_STATE, "assemble, set_dt, set_pulses or set_field_table first");
  tdde_status s = check_opts(c, o);
  if (s != TDDE_OK) return s;
  if (o->guess == TDDE_GUESS_GIVEN && !guess) return fail(c, TDDE_ERR_ARG, "GIVEN guess needs guess_dev");
  SolveArgs a = base_args(c, o);
  a.mode = MODE_STEP;
  a.psi = (double2*)psi;
  a.guess_in = (const double2*)guess;
  a.t0 = t;
  a.step0 = 0;
  a.n_steps = nullptr;
  if (split_serves(c, o)) {
    c->ones.assign((size_t)c->d.batch, 1);
    HIP_TRY(c, hipMemcpyAsync(c->n_steps_dev, c->ones.data(), (size_t)c->d.batch * sizeof(int), hipMemcpyHostToDevice,
                              c->stream));
    a.n_steps = c->n_steps_dev;
    if ((s = run_split(c, a)) != TDDE_OK) return s;
    if (!stats) return TDDE_OK;
    return collect_stats(c, stats, c->stats_dev, nullptr);
  }
  if ((s = run_persistent(c, a, 1)) != TDDE_OK) return s;
  if (!stats) return TDDE_OK;
  return collect_stats(c, stats);
}

tdde_status tdde_run_batched(tdde_ctx* c, void* psi, double t0, int32_t step0, int32_t n_chunk, const int32_t* n_steps,
                             const void* guess, const tdde_solve_opts* o, void* stats_dev) {
  if (!c || !psi || !n_steps) return fail(c, TDDE_ERR_ARG, "null argument");
  if (!c->assembled || !c->dt_set || !(c->pulses_set || c->use_table))
    return fail(c, TDDE_ERR_STATE, "assemble, set_dt, set_pulses or set_field_table first");
  tdde_status s = check_opts(c, o);
  if (s != TDDE_OK) return s;
  if (o->guess == TDDE_GUESS_GIVEN && (!guess || n_chunk != 1))
    return fail(c, TDDE_ERR_ARG, "a GIVEN guess needs guess_dev and n_chunk == 1");
  if (n_chunk <= 0 || n_chunk > 64 || step0 < 0) return fail(c, TDDE_ERR_ARG, "1 <= n_chunk <= 64, step0 >= 0");
  if (c->use_table)
    for (int b = 0; b < c->d.batch; ++b) {
      // rows of the steps this launch runs for instance b (the last one forms no further step's data)
      const long last = std::min<long>(n_steps[b], (long)step0 + n_chunk);
      if (last > step0 && last > c->ftab_rows)
        return fail(c, TDDE_ERR_ARG, "field table has no row for step " + std::to_string(last - 1));
    }
  HIP_TRY(c, hipMemcpyAsync(c->n_steps_dev, n_steps, (size_t)c->d.batch * sizeof(int), hipMemcpyHostToDevice, c->stream));
  SolveArgs a = base_args(c, o);
  a.mode = MODE_STEP;
  a.psi = (double2*)psi;
  a.t0 = t0;
  a.step0 = step0;
  a.n_chunk = n_chunk;
  a.n_steps = c->n_steps_dev;
  a.guess_in = (const double2*)guess;
  a.stats = (StatsDev*)stats_dev;
  if (split_serves(c, o)) return run_split(c, a);
  return run_persistent(c, a, n_chunk);
}


// ------------------------------------------------------------------------------------------ spectrum
// Photoelectron energy spectrum of eq. dPdE: dP/dE(E_n) = sum over channels |v_n^T S psi_j|^2 / dE_n
// with the caller's field-free eigenvectors v_n of the channel's radial block (box-normalised,
// v^T S v = 1), dE_n = (E_{n+1} - E_{n-1}) / 2, each channel's density interpolated linearly onto the
// energy grid (zero outside its levels) and summed in channel order.

// u_n = S v_n for every level (S of the block's kappa; copy when S = I).
__global__ void spec_sv_kernel(DevOp<double> op, const int* blk_kb, const int* lev0, int nblk, const double* v,
                               double* u) {
  const int nr = op.nr, nb = op.nb;
  const long total = (long)lev0[nblk] * 2 * nr;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long n = e / (2 * nr);
    const int q = (int)(e - n * 2 * nr), s = q / nr, i = q - s * nr;
    if (op.n_s == 0) { u[e] = v[e]; continue; }
    int b = 0;
    while (b + 1 < nblk && lev0[b + 1] <= n) ++b;
    const int kb = blk_kb[b];
    const double* vn = v + n * 2 * nr;
    double acc = 0.0;
    for (int s2 = 0; s2 < 2; ++s2) {
      if (!op.pq_s && s2 != s) continue;
      const double* band = op.s_blk + ((size_t)kb * 4 + s * 2 + s2) * nb * nr;
      for (int d = 0; d < nb; ++d) {
        const int i2 = i + d - op.hb;
        if (i2 >= 0 && i2 < nr) acc = fma(band[(size_t)d * nr + i], vn[(size_t)s2 * nr + i2], acc);
      }
    }
    u[e] = acc;
  }
}

// dens[b][j][k] = |u_{n}^T psi[b][j]|^2 / dE_n for the levels n = lev0[blk] + k of channel j's block.
// One work-group per (channel, instance); wave w takes levels k = w, w + 4, ...
__global__ __launch_bounds__(kThreads) void spec_project_kernel(const int* blk_of, const int* lev0, const double* Ebuf,
                                                               const double* u, const double2* psi, int nr, int nang,
                                                               int maxlev, double* dens) {
  const int j = blockIdx.x, b = blockIdx.y;
  const int blk = blk_of[j];
  const int n0 = lev0[blk], nl = lev0[blk + 1] - n0;
  const double* Eb = Ebuf + n0 + 2 * blk;  // Eb[0] level below, Eb[1 .. nl] levels, Eb[nl + 1] level above
  const double2* x = psi + ((size_t)b * nang + j) * 2 * nr;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = wave; k < nl; k += kThreads / 64) {
    const double* un = u + (size_t)(n0 + k) * 2 * nr;
    double re = 0.0, im = 0.0;
    for (int q = lane; q < 2 * nr; q += 64) {
      const double w = un[q];
      const double2 xv = x[q];
      re = fma(w, xv.x, re);
      im = fma(w, xv.y, im);
    }
    for (int off = 32; off > 0; off >>= 1) {
      re += __shfl_xor(re, off, 64);
      im += __shfl_xor(im, off, 64);
    }
    if (lane == 0) {
      const double dE = 0.5 * (Eb[k + 2] - Eb[k]);
      dens[((size_t)b * nang + j) * maxlev + k] = (re * re + im * im) / dE;
    }
  }
}

// dpde[b][g]: sum over channels (in order) of the linear interpolation of the channel's density at
// grid[g]; zero outside the channel's first and last level.
__global__ void spec_grid_kernel(const int* blk_of, const int* lev0, const double* Ebuf, const double* dens,
                                 const double* grid, int n_grid, int nang, int maxlev, int B, double* dpde) {
  const int total = B * n_grid;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int b = e / n_grid, g = e - b * n_grid;
    const double x = grid[g];
    double acc = 0.0;
    for (int j = 0; j < nang; ++j) {
      const int blk = blk_of[j];
      const int n0 = lev0[blk], nl = lev0[blk + 1] - n0;
      if (nl == 0) continue;
      const double* L = Ebuf + n0 + 2 * blk + 1;  // the block's levels, ascending
      if (x < L[0] || x > L[nl - 1]) continue;
      int lo = 0, hi = nl - 1;  // L[lo] <= x <= L[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (L[mid] <= x) lo = mid; else hi = mid;
      }
      const double* d = dens + ((size_t)b * nang + j) * maxlev;
      if (nl == 1) { acc += d[0]; continue; }
      const double t = (x - L[lo]) / (L[hi] - L[lo]);
      acc += d[lo] + t * (d[hi] - d[lo]);
    }
    dpde[e] = acc;
  }
}

// err[b] = sum_g (|p - q|^2 at g and g + 1, averaged) * (grid[g + 1] - grid[g]): the trapezoidal
// integral of the squared difference; one work-group per instance, fixed summation order.
__global__ __launch_bounds__(kThreads) void spec_error_kernel(const double* p, const double* q, const double* grid,
                                                             int n_grid, double* err) {
  __shared__ double red[2 * kThreads / 64];
  const int b = blockIdx.x;
  const double* pb = p + (size_t)b * n_grid;
  const double* qb = q + (size_t)b * n_grid;
  double acc = 0.0;
  for (int g = threadIdx.x; g + 1 < n_grid; g += kThreads) {
    const double d0 = pb[g] - qb[g], d1 = pb[g + 1] - qb[g + 1];
    acc += 0.5 * (d0 * d0 + d1 * d1) * (grid[g + 1] - grid[g]);
  }
  const double2 t = wg_sum2(make_double2(acc, 0.0), red);
  if (threadIdx.x == 0) err[b] = t.x;
}

tdde_status tdde_spectrum_setup(tdde_ctx* c, int32_t n_blk, const int32_t* blk_of, const int32_t* n_lev,
                                const double* levels, const double* edges, const double* vecs, const double* grid,
                                int32_t n_grid) {
  if (!c || !blk_of || !n_lev || !levels || !edges || !vecs || !grid) return fail(c, TDDE_ERR_ARG, "null argument");
  if (!c->assembled) return fail(c, TDDE_ERR_STATE, "assemble first");
  if (c->spec_set) return fail(c, TDDE_ERR_STATE, "spectrum already set up");
  if (c->has_chan) return fail(c, TDDE_ERR_ARG, "spectrum needs real kappa-polynomial blocks (no per-channel bands)");
  const int nang = c->d.nang, nr = c->d.nr;
  if (n_blk < 1 || n_grid < 2) return fail(c, TDDE_ERR_ARG, "n_blk >= 1 and n_grid >= 2 required");
  std::vector<int> kb_of_blk(n_blk, -1);
  for (int j = 0; j < nang; ++j) {
    if (blk_of[j] < 0 || blk_of[j] >= n_blk) return fail(c, TDDE_ERR_ARG, "block index out of range");
    if (kb_of_blk[blk_of[j]] < 0) kb_of_blk[blk_of[j]] = j;
    else if (c->kappa[kb_of_blk[blk_of[j]]] != c->kappa[j])
      return fail(c, TDDE_ERR_ARG, "channels of one eigen-block must share kappa");
  }
  std::vector<int> lev0(n_blk + 1, 0);
  int maxlev = 1;
  for (int b = 0; b < n_blk; ++b) {
    if (n_lev[b] < 0) return fail(c, TDDE_ERR_ARG, "negative level count");
    lev0[b + 1] = lev0[b] + n_lev[b];
    maxlev = std::max(maxlev, (int)n_lev[b]);
  }
  const int total = lev0[n_blk];
  std::vector<double> Ebuf((size_t)total + 2 * n_blk);
  for (int b = 0; b < n_blk; ++b) {
    double* dst = Ebuf.data() + lev0[b] + 2 * b;
    dst[0] = edges[2 * b];
    for (int k = 0; k < n_lev[b]; ++k) dst[1 + k] = levels[lev0[b] + k];
    dst[n_lev[b] + 1] = edges[2 * b + 1];
    for (int k = 0; k <= n_lev[b]; ++k)
      if (!(dst[k + 1] > dst[k])) return fail(c, TDDE_ERR_ARG, "levels (with the edges) must ascend strictly");
  }
  for (int g = 0; g + 1 < n_grid; ++g)
    if (!(grid[g + 1] > grid[g])) return fail(c, TDDE_ERR_ARG, "grid must ascend strictly");
  // the kappa block (distinct-kappa index of the operator) of each eigen-block
  std::vector<int> kblk(nang);
  {
    std::map<double, int> seen;
    for (int j = 0; j < nang; ++j) {
      auto it = seen.find(c->kappa[j]);
      if (it == seen.end()) it = seen.emplace(c->kappa[j], (int)seen.size()).first;
      kblk[j] = it->second;
    }
  }
  std::vector<int> blk_kb(n_blk, 0);
  for (int b = 0; b < n_blk; ++b) blk_kb[b] = kb_of_blk[b] >= 0 ? kblk[kb_of_blk[b]] : 0;
  tdde_status s;
  double* v_dev = nullptr;
  int* blk_kb_dev = nullptr;
  if ((s = upload(c, &c->spec_blk_of, blk_of, nang)) != TDDE_OK) return s;
  if ((s = upload(c, &c->spec_lev0, lev0.data(), lev0.size())) != TDDE_OK) return s;
  if ((s = upload(c, &blk_kb_dev, blk_kb.data(), blk_kb.size())) != TDDE_OK) return s;
  if ((s = upload(c, &c->spec_E, Ebuf.data(), Ebuf.size())) != TDDE_OK) return s;
  if ((s = upload(c, &v_dev, vecs, (size_t)total * 2 * nr)) != TDDE_OK) return s;
  if ((s = dev_alloc(c, &c->spec_U, (size_t)total * 2 * nr)) != TDDE_OK) return s;
  if ((s = upload(c, &c->spec_grid, grid, n_grid)) != TDDE_OK) return s;
  if ((s = dev_alloc(c, &c->spec_dens, (size_t)c->d.batch * nang * maxlev)) != TDDE_OK) return s;
  if ((s = dev_alloc(c, &c->spec_err, (size_t)c->d.batch)) != TDDE_OK) return s;
  if (total > 0) {
    hipLaunchKernelGGL(spec_sv_kernel, dim3(1024), dim3(256), 0, c->stream, c->op64, blk_kb_dev, c->spec_lev0, n_blk,
                       v_dev, c->spec_U);
    HIP_TRY(c, hipGetLastError());
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->spec_nblk = n_blk;
  c->spec_maxlev = maxlev;
  c->spec_ngrid = n_grid;
  c->spec_set = true;
  return TDDE_OK;
}

tdde_status tdde_spectrum(tdde_ctx* c, const void* psi, void* dpde) {
  if (!c || !psi || !dpde) return fail(c, TDDE_ERR_ARG, "null argument");
  if (!c->spec_set) return fail(c, TDDE_ERR_STATE, "tdde_spectrum_setup first");
  const int nang = c->d.nang, B = c->d.batch;
  hipLaunchKernelGGL(spec_project_kernel, dim3(nang, B), dim3(kThreads), 0, c->stream, c->spec_blk_of, c->spec_lev0,
                     c->spec_E, c->spec_U, (const double2*)psi, c->d.nr, nang, c->spec_maxlev, c->spec_dens);
  const int tot = B * c->spec_ngrid;
  hipLaunchKernelGGL(spec_grid_kernel, dim3((tot + 255) / 256), dim3(256), 0, c->stream, c->spec_blk_of, c->spec_lev0,
                     c->spec_E, c->spec_dens, c->spec_grid, c->spec_ngrid, nang, c->spec_maxlev, B, (double*)dpde);
  HIP_TRY(c, hipGetLastError());
  return TDDE_OK;
}

tdde_status tdde_spectrum_error(tdde_ctx* c, const void* p, const void* q, double* err) {
  if (!c || !p || !q || !err) return fail(c, TDDE_ERR_ARG, "null argument");
  if (!c->spec_set) return fail(c, TDDE_ERR_STATE, "tdde_spectrum_setup first");
  hipLaunchKernelGGL(spec_error_kernel, dim3(c->d.batch), dim3(kThreads), 0, c->stream, (const double*)p,
                     (const double*)q, c->spec_grid, c->spec_ngrid, c->spec_err);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipMemcpyAsync(err, c->spec_err, (size_t)c->d.batch * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return TDDE_OK;
}
