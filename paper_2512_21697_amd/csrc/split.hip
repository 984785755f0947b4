// Kernels of the kernel-per-window BiCGSTAB (split.hpp): the same iteration as the persistent
// solver, one kernel per window, scalar decisions taken by the last work-group of each instance.
#include "split.hpp"
#include "solver.hpp"

namespace tdde {

namespace {

// Launch-shape constants (compile-time knobs).
#ifndef TDDE_SPLIT_APPLY_WAVES
#define TDDE_SPLIT_APPLY_WAVES 2
#endif
#ifndef TDDE_SPLIT_GB
#define TDDE_SPLIT_GB 10  // half a 20-entry pattern row per batch: fewer registers, measured faster here
#endif
#ifndef TDDE_SPLIT_TR
#define TDDE_SPLIT_TR 1
#endif
// waves per SIMD asked of the apply kernels, their gather batch and coupling terms per tap round
constexpr int kSpWaves = TDDE_SPLIT_APPLY_WAVES;
constexpr int kSpGB = TDDE_SPLIT_GB;
constexpr int kSpTR = TDDE_SPLIT_TR;
#ifndef TDDE_SPLIT_CHAIN_AHEAD
#define TDDE_SPLIT_CHAIN_AHEAD 1
#endif
#ifndef TDDE_SPLIT_CHAIN_WAVES
#define TDDE_SPLIT_CHAIN_WAVES 2
#endif
#ifndef TDDE_SPLIT_CHAIN_AHEAD32
#define TDDE_SPLIT_CHAIN_AHEAD32 1
#endif
// rows of factor operands in flight per lane in the chain solves (FP64 factors; FP32 factors take half
// the registers per row), and the waves per SIMD asked of them
constexpr int kSpChainAhead = TDDE_SPLIT_CHAIN_AHEAD;
constexpr int kSpChainAhead32 = TDDE_SPLIT_CHAIN_AHEAD32;
constexpr int kSpChainWaves = TDDE_SPLIT_CHAIN_WAVES;

// Work-group -> (instance b, work-group g of the instance) for the apply and vector kernels of a
// B x G grid: w = 8 (B q + b) + x with g = 8 q + x, so work-group g of every instance runs on XCD
// g % 8 and takes tiles t = g, g + G, ... (tile_coords: a radial tile of all channels on one XCD).
struct SpWg {
  int b, g;
};
__device__ inline SpWg sp_wg(int B) {
  const int w = blockIdx.x;
  return {(w >> 3) % B, (w / (8 * B)) * 8 + (w & 7)};
}

// LDS of the reductions (every kernel with partials) and of the tile applies.
struct SpRed {
  double red[2 * kThreads / 64];
  int last;
};
struct SpLds {
  TileLds<double> tile;
  TermLds tl, tl2;
  SpRed r;
};

__device__ inline void sp_partial(const SplitArgs& a, const SpWg& w, int slot, double2 v, SpRed& L) {
  const double2 s = wg_sum2(v, L.red);
  if (threadIdx.x == 0) a.part[((size_t)w.b * a.G + w.g) * kSpSlots + slot] = s;
}

// Arrival of a work-group that has written its partials; true in the instance's last one, which then
// sees every partial of the instance. The counter is reset by that last arrival.
__device__ inline bool sp_last(const SplitArgs& a, const SpWg& w, SpRed& L) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int* c = a.cnt + (size_t)w.b * kSpCntLine;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const int old = __hip_atomic_fetch_add(c, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int last = old == a.G - 1;
    if (last) __hip_atomic_store(c, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    L.last = last;
  }
  __syncthreads();
  const bool last = L.last != 0;
  if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return last;
}

// Sum of one slot over the instance's G partials, work-group order then the fixed work-group sum.
__device__ inline double2 sp_total(const SplitArgs& a, int b, int slot, SpRed& L) {
  double2 acc = make_double2(0.0, 0.0);
  for (int g = threadIdx.x; g < a.G; g += kThreads) {
    const double2 v = a.part[((size_t)b * a.G + g) * kSpSlots + slot];
    acc.x += v.x;
    acc.y += v.y;
  }
  return wg_sum2(acc, L.red);
}

// Field values of `step` into a term table: row `step` of the field table, or the pulses at the
// step's midpoint (the persistent solver's values, bit for bit).
__device__ inline void sp_fields(const SplitArgs& a, int b, int step, TermLds& tl) {
  const PulseDev* pulses = a.pulses;
  terms_fields(a.op.n_terms, a.op.n_groups, tl, [&](int m) {
    const int fi = a.op.t_field[m];
    const double f = a.ftab != nullptr ? a.ftab[((size_t)b * a.ftab_rows + step) * a.n_fields + fi]
                                       : pulse_eval(pulses[(size_t)b * a.n_fields + fi], mid_time(a.t0, step, a.dt));
    const double2 c = a.op.t_coef[m];
    return make_double2(c.x * f, c.y * f);
  });
}

// Tiles of work-group g of instance b: f(element, S x, H x, H' x) for every owned element.
template <bool TWO, typename F>
__device__ inline void sp_tiles(const SplitArgs& a, const SpWg& w, const double2* xin, SpLds& L, F&& f) {
  const DevOp<double>& op = a.op;
  const int n_tiles = op.nang * op.n_itiles;
  const size_t base = (size_t)w.b * a.E;
  for (int t = w.g; t < n_tiles; t += a.G) {
    int j, it;
    tile_coords(op.nang, op.n_itiles, t, j, it);
    const SH<double> r = apply_tile<double, TWO, kSpGB, kSpTR>(op, xin + base, j, it * kTileR, L.tl, L.tile, &L.tl2);
    const long e = tile_elem(op.nr, j, it);
    if (e >= 0) f(base + e, r.sx, r.hx, r.hx2);
  }
}

// Elements of work-group g of instance b (vector kernels): g * 256 + thread, strided by G * 256.
template <typename F>
__device__ inline void sp_elems(const SplitArgs& a, const SpWg& w, F&& f) {
  const size_t base = (size_t)w.b * a.E;
  const size_t stride = (size_t)a.G * kThreads;
  for (size_t e = (size_t)w.g * kThreads + threadIdx.x; e < (size_t)a.E; e += stride) f(base + e);
}

// The same elements in batches of VB per thread: load(e) for the VB elements of a batch, then
// compute(e, loaded) in element order (per-thread order as in sp_elems), so that a thread has the
// loads of VB elements in flight at once.
template <int kVB, typename LD, typename CP>
__device__ inline void sp_elems_batched(const SplitArgs& a, const SpWg& w, LD&& load, CP&& compute) {
  const size_t base = (size_t)w.b * a.E;
  const size_t stride = (size_t)a.G * kThreads;
  size_t e = (size_t)w.g * kThreads + threadIdx.x;
  using V = decltype(load(size_t(0)));
  for (; e + (kVB - 1) * stride < (size_t)a.E; e += kVB * stride) {
    V v[kVB];
#pragma unroll
    for (int u = 0; u < kVB; ++u) v[u] = load(base + e + u * stride);
#pragma unroll
    for (int u = 0; u < kVB; ++u) compute(base + e + u * stride, v[u]);
  }
  for (; e < (size_t)a.E; e += stride) compute(base + e, load(base + e));
}

__device__ inline bool sp_next_exists(const SplitArgs& a, int b, const SplitCtl& c) {
  return c.k + 1 < a.n_chunk && c.step + 1 < a.n_steps[b];
}

// ---- decisions (thread 0 of the deciding work-group, on its copy of the control block)

// Statistics row of the finished step (status: the ABI's tdde_status value).
__device__ inline void sp_report(const SplitArgs& a, int b, const SplitCtl& c, int status) {
  if (a.stats == nullptr) return;
  StatsDev& o = static_cast<StatsDev*>(a.stats)[(size_t)c.k * a.B + b];
  o.status = status;
  o.iters = c.iters;
  o.matvecs = c.matvecs;
  o.restarts = c.restarts;
  o.outer_iters = 0;
  o.precs = c.precs;
  o.rel_res = c.rel_res;
  o.true_rel_res = c.true_rel_res;
}

// On to the next step (its per-step counters reset).
__device__ inline void sp_advance(SplitCtl& c) {
  c.step++;
  c.k++;
  c.iters = c.matvecs = c.restarts = c.precs = 0;
  c.nofuse = 0;
  c.fresh = 1;
  c.rho = c.alpha = c.omega = make_double2(1.0, 0.0);
  c.beta = make_double2(0.0, 0.0);
  c.rel_res = c.true_rel_res = 0.0;
}

// A step ends (any status): report it; the next step of the call, if any, forms its own data.
__device__ inline void sp_finish(const SplitArgs& a, int b, SplitCtl& c, int status) {
  sp_report(a, b, c, status);
  const bool next = sp_next_exists(a, b, c);
  sp_advance(c);
  c.state = next ? SP_INIT : SP_FINISHED;
}

// Start-of-iteration decision (the persistent solver's first window): rr = ||r||^2, rho = <r^, r>.
__device__ inline void sp_decide_w0(const SplitArgs& a, int b, SplitCtl& c, double2 rho, double rr) {
  c.rel_res = c.bb > 0 ? sqrt(rr / c.bb) : 0.0;
  const double rn = sqrt(rho.x * rho.x + rho.y * rho.y);
  if (!isfinite(rr) || !isfinite(c.bb) || !isfinite(rn)) {
    c.true_rel_res = c.rel_res;
    sp_finish(a, b, c, 3);  // TDDE_NONFINITE
  } else if (rr <= c.target2) {
    c.state = SP_VERIFY;
  } else if (c.iters >= a.max_iter) {
    sp_finish(a, b, c, 1);  // TDDE_NOT_CONVERGED
  } else {
    const double om = sqrt(c.omega.x * c.omega.x + c.omega.y * c.omega.y);
    if (rn <= 1e-300 * (1.0 + rr) || (!c.fresh && om == 0.0)) {
      // rho or omega vanished: restart from the same r with r^ = r
      c.restarts++;
      if (c.restarts > 20) sp_finish(a, b, c, 2);  // TDDE_BREAKDOWN
      else c.state = SP_RESTART;
    } else {
      if (!c.fresh) c.beta = dmul(cdiv(rho, c.rho), cdiv(c.alpha, c.omega));
      c.rho = rho;
      c.state = SP_ACTIVE;
    }
  }
}

// First decision of a step whose b, r, r^ are formed: bb = ||b||^2, rr = ||r||^2 = <r^, r>.
__device__ inline void sp_begin_step(const SplitArgs& a, int b, SplitCtl& c, double bb, double rr) {
  c.bb = bb;
  c.target2 = a.tol * a.tol * bb;
  c.fresh = 1;
  sp_decide_w0(a, b, c, make_double2(rr, 0.0), rr);
}

// ---- kernels




__global__ void sp_begin_kernel(SplitArgs a) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.B) return;
  SplitCtl c{};
  c.step = a.step0;
  c.k = 0;
  c.fresh = 1;
  c.rho = c.alpha = c.omega = make_double2(1.0, 0.0);
  c.state = a.step0 < a.n_steps[b] ? SP_INIT : SP_FINISHED;
  a.ctl[b] = c;
  a.cnt[(size_t)b * kSpCntLine] = 0;
}

// INIT: right-hand side and initial residual of the step; RESTART: r^ = r and ||r||^2.
__global__ __attribute__((amdgpu_flat_work_group_size(kThreads, kThreads), amdgpu_waves_per_eu(kSpWaves)))
void sp_prologue_kernel(SplitArgs a) {
  __shared__ SpLds L;
  SpRed& R = L.r;
  const SpWg w = sp_wg(a.B);
  const SplitCtl c = a.ctl[w.b];
  if (c.state == SP_INIT) {
    terms_layout<double>(a.op, L.tl);
    sp_fields(a, w.b, c.step, L.tl);
    double2* bv = a.bvec[c.par];
    const double2 mahc = make_double2(0.0, -0.5 * a.dt), mdt = make_double2(0.0, -a.dt);
    double2 bb = make_double2(0.0, 0.0), rr = bb;
    sp_tiles<false>(a, w, a.x, L, [&](size_t e, double2 sx, double2 hx, double2) {
      const double2 bval = cfma<double>(mahc, hx, sx);
      bv[e] = bval;
      dot_acc(bb, bval, bval);
      const double2 rv = cmul<double>(mdt, hx);  // b - A psi = -i dt H psi
      a.r[e] = rv;
      a.rh[e] = rv;
      dot_acc(rr, rv, rv);
    });
    sp_partial(a, w, SPS_A, bb, R);
    sp_partial(a, w, SPS_B, rr, R);
    if (!sp_last(a, w, R)) return;
    const double bbt = sp_total(a, w.b, SPS_A, R).x, rrt = sp_total(a, w.b, SPS_B, R).x;
    if (threadIdx.x == 0) {
      SplitCtl n = c;
      n.matvecs = 1;
      sp_begin_step(a, w.b, n, bbt, rrt);
      a.ctl[w.b] = n;
    }
  } else if (c.state == SP_RESTART) {
    double2 rr = make_double2(0.0, 0.0);
    sp_elems(a, w, [&](size_t e) {
      const double2 rv = a.r[e];
      a.rh[e] = rv;
      dot_acc(rr, rv, rv);
    });
    sp_partial(a, w, SPS_A, rr, R);
    if (!sp_last(a, w, R)) return;
    const double rrt = sp_total(a, w.b, SPS_A, R).x;
    if (threadIdx.x == 0) {
      SplitCtl n = c;
      n.fresh = 1;
      sp_decide_w0(a, w.b, n, make_double2(rrt, 0.0), rrt);
      a.ctl[w.b] = n;
    }
  }
}

// Chain work item of a work-group (the channels of one factor block, items of a block on one XCD):
// instance vectors and channel list; 0 channels for a padding item.
__device__ inline int sp_item(const SplitArgs& a, int b, double2* in, double2* out, double2 c1, double2 c2,
                              ChainIO<double>& io, const int*& js) {
  const int nk = chain_item(a.pc, blockIdx.x, js);
  const size_t ib = (size_t)b * a.E;
  io.r = a.r + ib;
  io.v = a.v + ib;
  io.pz = in + ib;
  io.out = out + ib;
  io.c1 = c1;
  io.c2 = c2;
  return nk;
}

// p = r (new cycle) or r + beta (p - omega v), p^ = K^-1 p: one chain work item per work-group.
__global__ __attribute__((amdgpu_flat_work_group_size(kThreads, kThreads), amdgpu_waves_per_eu(kSpChainWaves)))
void sp_dir_chain_kernel(SplitArgs a) {
  __shared__ ChainLds<double> L;
  const int b = blockIdx.y;
  const SplitCtl c = a.ctl[b];
  if (c.state != SP_ACTIVE) return;
  ChainIO<double> io;
  const int* js = nullptr;
  const int nk = sp_item(a, b, a.p, a.ph, c.beta, c.omega, io, js);
  if (nk == 0) return;
  const int blk = a.pc.block_of[js[0]];
  if (a.prec32) {
    if (c.fresh) chain_solve<double, MODE_FRESH, kSpChainAhead32, float>(a.pc32, blk, a.op.nr, io, js, nk, L);
    else chain_solve<double, MODE_P, kSpChainAhead32, float>(a.pc32, blk, a.op.nr, io, js, nk, L);
  } else {
    if (c.fresh) chain_solve<double, MODE_FRESH, kSpChainAhead>(a.pc, blk, a.op.nr, io, js, nk, L);
    else chain_solve<double, MODE_P, kSpChainAhead>(a.pc, blk, a.op.nr, io, js, nk, L);
  }
}

// Without the preconditioner: p = r or r + beta (p - omega v).
__global__ __launch_bounds__(kThreads) void sp_dir_plain_kernel(SplitArgs a) {
  const SpWg w = sp_wg(a.B);
  const SplitCtl c = a.ctl[w.b];
  if (c.state != SP_ACTIVE) return;
  const double2 beta = c.beta, omega = c.omega;
  const bool fr = c.fresh != 0;
  sp_elems(a, w, [&](size_t e) {
    const double2 rv = a.r[e];
    a.p[e] = fr ? rv : cfma<double>(beta, csub<double>(a.p[e], cmul<double>(omega, a.v[e])), rv);
  });
}

// v = A p^, <r^, v> -> alpha (or a restart when it vanishes).
__global__ __attribute__((amdgpu_flat_work_group_size(kThreads, kThreads), amdgpu_waves_per_eu(kSpWaves)))
void sp_apply_v_kernel(SplitArgs a) {
  __shared__ SpLds L;
  SpRed& R = L.r;
  const SpWg w = sp_wg(a.B);
  const SplitCtl c = a.ctl[w.b];
  if (c.state != SP_ACTIVE) return;
  terms_layout<double>(a.op, L.tl);
  sp_fields(a, w.b, c.step, L.tl);
  const double2 ahc = make_double2(0.0, 0.5 * a.dt);
  double2 acc = make_double2(0.0, 0.0);
  sp_tiles<false>(a, w, a.ph, L, [&](size_t e, double2 sx, double2 hx, double2) {
    const double2 vv = cfma<double>(ahc, hx, sx);
    a.v[e] = vv;
    dot_acc(acc, a.rh[e], vv);
  });
  sp_partial(a, w, SPS_A, acc, R);
  if (!sp_last(a, w, R)) return;
  const double2 rv = sp_total(a, w.b, SPS_A, R);
  if (threadIdx.x == 0) {
    SplitCtl n = c;
    n.matvecs++;
    if (a.use_prec) n.precs++;  // p^ of this iteration
    n.fresh = 0;
    if (rv.x == 0.0 && rv.y == 0.0) {
      n.restarts++;
      n.state = SP_RESTART;
    } else {
      n.alpha = cdiv(n.rho, rv);
    }
    a.ctl[w.b] = n;
  }
}

// s = r - alpha v, ||s||^2 -> half-step test.
__global__ __launch_bounds__(kThreads) void sp_s_kernel(SplitArgs a) {
  __shared__ SpRed R;
  const SpWg w = sp_wg(a.B);
  const SplitCtl c = a.ctl[w.b];
  if (c.state != SP_ACTIVE) return;
  const double2 al = c.alpha;
  double n2 = 0.0;
  struct RV { double2 r, v; };
  sp_elems_batched<4>(
      a, w, [&](size_t e) { return RV{gld(a.r + e), gld(a.v + e)}; },
      [&](size_t e, RV q) {
        const double2 sv = csub<double>(q.r, cmul<double>(al, q.v));
        gst(a.s + e, sv);
        n2 += sv.x * sv.x + sv.y * sv.y;
      });
  sp_partial(a, w, SPS_A, make_double2(n2, 0.0), R);
  if (!sp_last(a, w, R)) return;
  const double ss = sp_total(a, w.b, SPS_A, R).x;
  if (threadIdx.x == 0 && ss <= c.target2) {
    SplitCtl n = c;
    n.iters++;
    n.rel_res = n.bb > 0 ? sqrt(ss / n.bb) : 0.0;
    n.state = SP_HALF;
    a.ctl[w.b] = n;
  }
}

// s^ = K^-1 s.
__global__ __attribute__((amdgpu_flat_work_group_size(kThreads, kThreads), amdgpu_waves_per_eu(kSpChainWaves)))
void sp_chain_s_kernel(SplitArgs a) {
  __shared__ ChainLds<double> L;
  const int b = blockIdx.y;
  const SplitCtl c = a.ctl[b];
  if (c.state != SP_ACTIVE) return;
  ChainIO<double> io;
  const int* js = nullptr;
  const int nk = sp_item(a, b, a.s, a.sh, c.alpha, c.alpha, io, js);
  if (nk == 0) return;
  if (a.prec32) chain_solve<double, MODE_IN_S, kSpChainAhead32, float>(a.pc32, a.pc.block_of[js[0]], a.op.nr, io, js, nk, L);
  else chain_solve<double, MODE_IN_S, kSpChainAhead>(a.pc, a.pc.block_of[js[0]], a.op.nr, io, js, nk, L);
}

// t = A s^, <t, s>, <t, t> -> omega.
__global__ __attribute__((amdgpu_flat_work_group_size(kThreads, kThreads), amdgpu_waves_per_eu(kSpWaves)))
void sp_apply_t_kernel(SplitArgs a) {
  __shared__ SpLds L;
  SpRed& R = L.r;
  const SpWg w = sp_wg(a.B);
  const SplitCtl c = a.ctl[w.b];
  if (c.state != SP_ACTIVE) return;
  terms_layout<double>(a.op, L.tl);
  sp_fields(a, w.b, c.step, L.tl);
  const double2 ahc = make_double2(0.0, 0.5 * a.dt);
  double2 ts = make_double2(0.0, 0.0), tt = ts;
  sp_tiles<false>(a, w, a.sh, L, [&](size_t e, double2 sx, double2 hx, double2) {
    const double2 tv = cfma<double>(ahc, hx, sx);
    a.t[e] = tv;
    dot_acc(ts, tv, a.s[e]);
    dot_acc(tt, tv, tv);
  });
  sp_partial(a, w, SPS_A, ts, R);
  sp_partial(a, w, SPS_B, tt, R);
  if (!sp_last(a, w, R)) return;
  const double2 tst = sp_total(a, w.b, SPS_A, R);
  const double ttt = sp_total(a, w.b, SPS_B, R).x;
  if (threadIdx.x == 0) {
    SplitCtl n = c;
    n.matvecs++;
    if (a.use_prec) n.precs++;  // s^ of this iteration
    n.omega = ttt > 0.0 ? make_double2(tst.x / ttt, tst.y / ttt) : make_double2(0.0, 0.0);
    a.ctl[w.b] = n;
  }
}

// ACTIVE: x += alpha p^ + omega s^, r = s - omega t, <r^, r>, ||r||^2 -> next iteration's decision.
// HALF: x += alpha p^ (the half step ended the solve; the check follows).
__global__ __launch_bounds__(kThreads) void sp_xr_kernel(SplitArgs a) {
  __shared__ SpRed R;
  const SpWg w = sp_wg(a.B);
  const SplitCtl c = a.ctl[w.b];
  const double2 al = c.alpha;
  if (c.state == SP_HALF) {
    struct XP { double2 x, ph; };
    sp_elems_batched<4>(
        a, w, [&](size_t e) { return XP{gld(a.x + e), gld(a.ph + e)}; },
        [&](size_t e, XP q) { gst(a.x + e, cfma<double>(al, q.ph, q.x)); });
    return;
  }
  if (c.state != SP_ACTIVE) return;
  const double2 om = c.omega;
  double2 rho = make_double2(0.0, 0.0), rr = rho;
  struct XR { double2 x, ph, sh, s, t, rh; };
  sp_elems_batched<2>(
      a, w,
      [&](size_t e) { return XR{gld(a.x + e), gld(a.ph + e), gld(a.sh + e), gld(a.s + e), gld(a.t + e), gld(a.rh + e)}; },
      [&](size_t e, XR q) {
        gst(a.x + e, cfma<double>(om, q.sh, cfma<double>(al, q.ph, q.x)));
        const double2 rv = csub<double>(q.s, cmul<double>(om, q.t));
        gst(a.r + e, rv);
        dot_acc(rho, q.rh, rv);
        dot_acc(rr, rv, rv);
      });
  sp_partial(a, w, SPS_A, rho, R);
  sp_partial(a, w, SPS_B, rr, R);
  if (!sp_last(a, w, R)) return;
  const double2 rhot = sp_total(a, w.b, SPS_A, R);
  const double rrt = sp_total(a, w.b, SPS_B, R).x;
  if (threadIdx.x == 0) {
    SplitCtl n = c;
    n.iters++;
    sp_decide_w0(a, w.b, n, rhot, rrt);
    a.ctl[w.b] = n;
  }
}

// True residual of the step, fused with the next step's right-hand side and initial residual when
// the next step of the call follows (and no fused check of this step has failed yet).
__global__ __attribute__((amdgpu_flat_work_group_size(kThreads, kThreads), amdgpu_waves_per_eu(kSpWaves)))
void sp_check_kernel(SplitArgs a) {
  __shared__ SpLds L;
  SpRed& R = L.r;
  const SpWg w = sp_wg(a.B);
  const SplitCtl c = a.ctl[w.b];
  if (c.state != SP_HALF && c.state != SP_VERIFY && c.state != SP_VERIFY_NF) return;
  const bool fuse = c.state != SP_VERIFY_NF && !c.nofuse && sp_next_exists(a, w.b, c);
  terms_layout<double>(a.op, L.tl);
  sp_fields(a, w.b, c.step, L.tl);
  const double2 ahc = make_double2(0.0, 0.5 * a.dt), mahc = make_double2(0.0, -0.5 * a.dt),
                mdt = make_double2(0.0, -a.dt);
  const double2* bv = a.bvec[c.par];
  double2 acc = make_double2(0.0, 0.0);
  if (fuse) {
    terms_layout<double>(a.op, L.tl2);
    sp_fields(a, w.b, c.step + 1, L.tl2);
    double2* bn = a.bvec[c.par ^ 1];
    double2 accb = make_double2(0.0, 0.0), accr = accb;
    sp_tiles<true>(a, w, a.x, L, [&](size_t e, double2 sx, double2 hx, double2 hx2) {
      const double2 rt = csub<double>(bv[e], cfma<double>(ahc, hx, sx));
      dot_acc(acc, rt, rt);
      const double2 bval = cfma<double>(mahc, hx2, sx);
      bn[e] = bval;
      dot_acc(accb, bval, bval);
      const double2 rv = cmul<double>(mdt, hx2);  // b' - A' x = -i dt H' x
      a.r[e] = rv;
      a.rh[e] = rv;
      dot_acc(accr, rv, rv);
    });
    sp_partial(a, w, SPS_A, acc, R);
    sp_partial(a, w, SPS_B, accb, R);
    sp_partial(a, w, SPS_C, accr, R);
  } else {
    sp_tiles<false>(a, w, a.x, L, [&](size_t e, double2 sx, double2 hx, double2) {
      const double2 rt = csub<double>(bv[e], cfma<double>(ahc, hx, sx));
      a.r[e] = rt;
      dot_acc(acc, rt, rt);
    });
    sp_partial(a, w, SPS_A, acc, R);
  }
  if (!sp_last(a, w, R)) return;
  const double rr = sp_total(a, w.b, SPS_A, R).x;
  double nbb = 0.0, nrr = 0.0;
  if (fuse) {
    nbb = sp_total(a, w.b, SPS_B, R).x;
    nrr = sp_total(a, w.b, SPS_C, R).x;
  }
  if (threadIdx.x == 0) {
    SplitCtl n = c;
    n.matvecs++;
    n.true_rel_res = n.bb > 0 ? sqrt(rr / n.bb) : 0.0;
    if (rr <= n.target2) {
      sp_report(a, w.b, n, 0);
      if (fuse) {
        sp_advance(n);
        n.par ^= 1;
        sp_begin_step(a, w.b, n, nbb, nrr);
      } else {
        const bool next = sp_next_exists(a, w.b, n);
        sp_advance(n);
        n.state = next ? SP_INIT : SP_FINISHED;
      }
    } else if (n.iters >= a.max_iter) {
      sp_finish(a, w.b, n, 1);
    } else if (fuse) {
      n.nofuse = 1;  // r now holds the next step's residual: form this step's again, then restart
      n.state = SP_VERIFY_NF;
    } else {
      n.restarts++;  // the true residual is too large: restart from it
      n.state = SP_RESTART;
    }
    a.ctl[w.b] = n;
  }
}

// Unfinished instances into the host-visible flag of this block's parity.
__global__ void sp_sync_kernel(SplitArgs a, int parity) {
  __shared__ int n;
  if (threadIdx.x == 0) n = 0;
  __syncthreads();
  int mine = 0;
  for (int b = threadIdx.x; b < a.B; b += blockDim.x) mine += a.ctl[b].state != SP_FINISHED ? 1 : 0;
  if (mine) atomicAdd(&n, mine);
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(a.host_flag + parity, n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

}  // namespace

hipError_t split_launch_block(const SplitArgs& a, hipStream_t stream, int parity, bool first, const hipEvent_t* ev_v) {
  const dim3 blk(kThreads);
  const dim3 flat((unsigned)(a.B * a.G));
  const dim3 chains((unsigned)a.pc.n_items, (unsigned)a.B);
  if (first) hipLaunchKernelGGL(sp_begin_kernel, dim3((a.B + kThreads - 1) / kThreads), blk, 0, stream, a);
  hipLaunchKernelGGL(sp_prologue_kernel, flat, blk, 0, stream, a);
  if (a.use_prec) hipLaunchKernelGGL(sp_dir_chain_kernel, chains, blk, 0, stream, a);
  else hipLaunchKernelGGL(sp_dir_plain_kernel, flat, blk, 0, stream, a);
  if (ev_v != nullptr) {
    const hipError_t e = hipEventRecord(ev_v[0], stream);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(sp_apply_v_kernel, flat, blk, 0, stream, a);
  if (ev_v != nullptr) {
    const hipError_t e = hipEventRecord(ev_v[1], stream);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(sp_s_kernel, flat, blk, 0, stream, a);
  if (a.use_prec) hipLaunchKernelGGL(sp_chain_s_kernel, chains, blk, 0, stream, a);
  hipLaunchKernelGGL(sp_apply_t_kernel, flat, blk, 0, stream, a);
  hipLaunchKernelGGL(sp_xr_kernel, flat, blk, 0, stream, a);
  hipLaunchKernelGGL(sp_check_kernel, flat, blk, 0, stream, a);
  hipLaunchKernelGGL(sp_sync_kernel, dim3(1), blk, 0, stream, a, parity);
  return hipGetLastError();
}

}  // namespace tdde
