// Persistent BiCGSTAB for the Crank-Nicolson step (eq. solPsi), all instances of a batch in one
// cooperative launch.
//
// Grid: n_wg co-resident work-groups; instance b owns work-groups [b*G, (b+1)*G). Tiles
// (channel j, radial tile) of an instance are dealt round-robin to its G work-groups, so tile k
// runs on XCD (b*G + k % G) % 8: for G a multiple of 8 the same tile of every instance shares
// one L2 (operator bands are reused across instances), and for one instance all channels of a
// radial tile share one L2 (angular gathers hit in L2).
//
// Reductions are deterministic: every work-group writes one partial per dot product, and after
// the grid barrier every work-group of the instance sums the G partials in the same order.
// Each BiCGSTAB iteration (van der Vorst 1992; right preconditioner K = M of eq. matrixM when
// enabled) runs in five windows separated by grid barriers:
//   W0  rho, ||r|| -> convergence / restart decision, beta;  p = r + beta (p - omega v), p^ = K^-1 p
//   W1  v = A p^, <r^, v>
//   W2  alpha;  s = r - alpha v, ||s||  (and x + alpha p^ into the other iterate buffer when this
//       half step is expected to end the solve)
//   W3  ||s|| test (half step);  without preconditioner t = A s, <t, s>, <t, t>; with it s^ = K^-1 s
//   W3b (preconditioned only) t = A s^, <t, s>, <t, t>
//   W4  omega;  x += alpha p^ + omega s^,  r = s - omega t,  <r^, r>, ||r||
// The true-residual check (VERIFY / VCHECK states) runs in whichever windows follow convergence;
// when the half step ends the solve with x + alpha p^ already formed, it runs in W3 itself. The loop
// ends at the first barrier after which the count of unfinished work-groups is zero.
#pragma once
#include "apply.hpp"
#include "precond.hpp"

namespace tdde {

// ST_VERIFY: the true residual b - A x is formed in the next window; ST_VCHECK: it is tested in the
// window after that (accept, or restart from it as ST_PENDING, which the next W0 picks up).
enum { ST_INACTIVE = 0, ST_ACTIVE = 1, ST_VERIFY = 2, ST_DONE = 3, ST_FAILED = 4, ST_PENDING = 5, ST_BREAKDOWN = 6,
       ST_VCHECK = 7, ST_NONFINITE = 8 };
// Status reported for a final state (the ABI's tdde_status values).
__device__ inline int status_of(int state) {
  return state == ST_DONE ? 0 : (state == ST_BREAKDOWN ? 2 : (state == ST_NONFINITE ? 3 : 1));
}
// A slot is never read and written in the same barrier window by one instance.
//   RHO, RR: written W4, read W0; RR also written by a residual check and read in the window after it
//   AUX: ||r||^2 of a restart, written by a restart or a non-fused residual check, read W0 when PENDING
//   ORR, OBB: outer refinement residual / rhs norms (mixed precision)
// SLOT_N*: the next step's initial partials, formed with the residual check of the current step
enum { SLOT_RHO = 0, SLOT_RR, SLOT_RV, SLOT_SS, SLOT_TS, SLOT_TT, SLOT_BB, SLOT_AUX, SLOT_ORR, SLOT_OBB, SLOT_NRHO,
       SLOT_NRR, SLOT_NBB, kSlots };
enum { GUESS_ZERO = 0, GUESS_PREV = 1, GUESS_GIVEN = 2 };
enum { MODE_SOLVE = 0, MODE_STEP = 1 };

struct StatsDev {
  int status, iters, matvecs, restarts, outer_iters, precs;
  double rel_res, true_rel_res;
};

template <typename T> struct KVec {
  c2_t<T> *x, *r, *rh, *p, *ph, *v, *s, *sh, *t;
};

struct SolveArgs {
  DevOp<double> op64;
  DevOp<float> op32;
  DevPrec<double> pc64;
  DevPrec<float> pc32;
  KVec<double> v64;
  KVec<float> v32;
  double2* bvec;          // right-hand side workspace (FP64), even steps of a launch
  double2* bvec2;         // right-hand side of odd steps (the next step's is formed during this one)
  double2* xalt;          // second iterate buffer: x + alpha p^ formed with s, ahead of the half-step test
  double2* r64;           // outer residual (mixed precision)
  float2* rhs32;          // inner right-hand side (mixed precision)
  int B, G, E, n_wg;
  int mode, guess, use_prec, mixed;
  int max_iter, max_outer;
  double tol, inner_tol, dt, t0;
  int step0, n_chunk, n_fields, pad0;
  const int* n_steps;     // device [B] or null
  const PulseDev* pulses; // device [B][n_fields]
  const double* ftab;     // device [B][ftab_rows][n_fields] field table (MODE_STEP; null: the pulses)
  int ftab_rows, pad1;
  const double* fvals;    // device [B][n_fields]
  double2* psi;           // MODE_STEP state (in/out)
  const double2* guess_in;
  const double2* b_in;    // MODE_SOLVE right-hand side
  const double2* shadow;  // MODE_SOLVE: shadow residual r^ of the first cycle (null: r^ = r)
  double2* x_io;          // MODE_SOLVE solution (in: guess)
  double2* part;          // [B][G][kSlots]
  unsigned* bar;          // grid barrier state
  int* counters;          // [n_chunk][kCounterPerStep]
  StatsDev* stats;        // [n_chunk][B] or null
  unsigned long long* marks;  // optional phase timestamps of work-group 0: (wall clock << 8) | phase
  int n_marks;
};

// Phase timestamps (work-group 0, thread 0 only): the timing breakdown of a persistent launch.
struct Marks {
  unsigned long long* p;
  int n, cap;
  __device__ inline void mark(int id) {
    if (p != nullptr && blockIdx.x == 0 && threadIdx.x == 0 && n < cap) p[n++] = (wall_clock64() << 8) | (unsigned)id;
  }
};
constexpr int kCounterPerStep = 64;

struct WgInfo {
  int b, g, G, live;
};

struct Inst {
  int state, fresh, iters, matvecs, restarts, first, precs;
  int fused;       // the pending residual check also formed the next step's b, r, r^ and partials
  int nofuse;      // a failed check: form only the true residual from now on
  int next_ready;  // finished with the next step's initial data in place
  int xsel;        // the iterate lives in the second buffer
  int xahead;      // the other buffer holds x + alpha p^ of this iteration
  int spec_it;     // iteration whose half step is expected to end the solve (x + alpha p^ formed ahead)
  double2 rho, alpha, omega;
  double bb, target2, rel_res, true_rel_res;
};

template <typename T> union SharedLds {
  TileLds<T> tile;
  ChainLds<T> chain;
};

struct Shared {
  union {
    SharedLds<double> d;
    SharedLds<float> f;
  } u;
  double red[2 * kThreads / 64];
  TermLds tl;
  TermLds tl2;  // fields of the next step (formed with the current step's residual check)
};

__device__ inline void put_partial(const SolveArgs& a, const WgInfo& wi, int slot, double2 v, Shared& sh) {
  const double2 s = wg_sum2(v, sh.red);
  if (threadIdx.x == 0) a.part[((size_t)wi.b * wi.G + wi.g) * kSlots + slot] = s;
}
// Three slots at once (one round of partial loads).
__device__ inline void get_totals3(const SolveArgs& a, const WgInfo& wi, int s0, int s1, int s2, double2& t0,
                                   double2& t1, double2& t2, Shared& sh) {
  double2 a0 = make_double2(0.0, 0.0), a1 = a0, a2 = a0;
  for (int gg = threadIdx.x; gg < wi.G; gg += kThreads) {
    const double2* p = a.part + ((size_t)wi.b * wi.G + gg) * kSlots;
    const double2 v0 = p[s0], v1 = p[s1], v2 = p[s2];
    a0.x += v0.x; a0.y += v0.y;
    a1.x += v1.x; a1.y += v1.y;
    a2.x += v2.x; a2.y += v2.y;
  }
  t0 = wg_sum2(a0, sh.red);
  t1 = wg_sum2(a1, sh.red);
  t2 = wg_sum2(a2, sh.red);
}

__device__ inline double2 get_total(const SolveArgs& a, const WgInfo& wi, int slot, Shared& sh) {
  double2 acc = make_double2(0.0, 0.0);
  for (int gg = threadIdx.x; gg < wi.G; gg += kThreads) {
    const double2 v = a.part[((size_t)wi.b * wi.G + gg) * kSlots + slot];
    acc.x += v.x; acc.y += v.y;
  }
  return wg_sum2(acc, sh.red);
}

__device__ inline void counter_add(int* c, int v) {
  if (threadIdx.x == 0) __hip_atomic_fetch_add(c, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T> __device__ inline const DevOp<T>& op_of(const SolveArgs& a);
template <> __device__ inline const DevOp<double>& op_of<double>(const SolveArgs& a) { return a.op64; }
template <> __device__ inline const DevOp<float>& op_of<float>(const SolveArgs& a) { return a.op32; }
template <typename T> __device__ inline const DevPrec<T>& pc_of(const SolveArgs& a);
template <> __device__ inline const DevPrec<double>& pc_of<double>(const SolveArgs& a) { return a.pc64; }
template <> __device__ inline const DevPrec<float>& pc_of<float>(const SolveArgs& a) { return a.pc32; }
template <typename T> __device__ inline SharedLds<T>& lds_of(Shared& sh);
template <> __device__ inline SharedLds<double>& lds_of<double>(Shared& sh) { return sh.u.d; }
template <> __device__ inline SharedLds<float>& lds_of<float>(Shared& sh) { return sh.u.f; }

// Tile loop of the calling work-group over its instance (tiles t = g, g + G, ...; tile_coords).
#define FOR_TILES(op, wi)                                                              \
  for (int tile_ = (wi).g; tile_ < (op).nang * (op).n_itiles; tile_ += (wi).G)         \
    for (int j_ = 0, it_ = 0, once_ = (tile_coords((op).nang, (op).n_itiles, tile_, j_, it_), 1); once_; once_ = 0) \
      for (int i0_ = it_ * kTileR, once2_ = 1; once2_; once2_ = 0)

// Element owned by the calling thread in tile (j, i0); -1 for halo threads and points past nr.
template <typename T> __device__ inline long tile_elem(const DevOp<T>& op, int j, int i0) {
  return tile_elem(op.nr, j, i0 / kTileR);
}

// Chain loop: work item w of the chain order (the channels of one factor block solved together,
// items of one block on one XCD) is taken by work-group w mod G; padding items have no channel.
#define FOR_CHAINS(pc, wi)                                                   \
  for (int w_ = (wi).g; w_ < (pc).n_items; w_ += (wi).G)                   \
    for (const int* js_ = (pc).chain_order + (size_t)w_ * (pc).nc; js_ != nullptr; js_ = nullptr)       \
      for (int nk_ = chain_item(pc, w_, js_), once_ = 1; once_ && nk_ > 0; once_ = 0)

template <typename T>
__device__ inline c2_t<T> load_c(const c2_t<T>* p, long e) { return p[e]; }

// y = S x + ah * H x for own tiles of instance b (A of the step), with optional fused outputs.
// The caller supplies a functor on (element, S x, H x).
// GB: neighbour loads of a gather issued together (more registers, fewer round trips).
template <typename T, int GB = kGatherBatch, int TR = 2, typename F>
__device__ inline void apply_own(const SolveArgs& a, const WgInfo& wi, const c2_t<T>* xin, Shared& sh, F&& f) {
  const DevOp<T>& op = op_of<T>(a);
  FOR_TILES(op, wi) {
    SH<T> r = apply_tile<T, false, GB, TR>(op, xin, j_, i0_, sh.tl, lds_of<T>(sh).tile);
    const long e = tile_elem<T>(op, j_, i0_);
    if (e >= 0) f(e, r.sx, r.hx);
  }
}

// Same with the next step's fields as well: f(e, S x, H x, H_next x).
template <typename T, int GB = kGatherBatch, int TR = 2, typename F>
__device__ inline void apply_own2(const SolveArgs& a, const WgInfo& wi, const c2_t<T>* xin, Shared& sh, F&& f) {
  const DevOp<T>& op = op_of<T>(a);
  FOR_TILES(op, wi) {
    SH<T> r = apply_tile<T, true, GB, TR>(op, xin, j_, i0_, sh.tl, lds_of<T>(sh).tile, &sh.tl2);
    const long e = tile_elem<T>(op, j_, i0_);
    if (e >= 0) f(e, r.sx, r.hx, r.hx2);
  }
}

template <typename T, typename F>
__device__ inline void elem_own(const SolveArgs& a, const WgInfo& wi, F&& f) {
  const DevOp<T>& op = op_of<T>(a);
  FOR_TILES(op, wi) {
    const long e = tile_elem<T>(op, j_, i0_);
    if (e >= 0) f(e);
  }
}

template <typename T> __device__ inline c2_t<T> to_c(double2 z) { return cmk<T>((T)z.x, (T)z.y); }

__device__ inline double2 cdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ inline double2 dmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

// Preconditioner chain phase for own work items (MODE_P / MODE_FRESH / MODE_IN_S); the whole
// work-group solves one item (the channels of one factor block) at a time.
template <typename T, int MODE>
__device__ inline void chains_own(const SolveArgs& a, const WgInfo& wi, const KVec<T>& V, size_t base, double2 c1,
                                  double2 c2, Shared& sh) {
  const DevOp<T>& op = op_of<T>(a);
  const DevPrec<T>& pc = pc_of<T>(a);
  FOR_CHAINS(pc, wi) {
    ChainIO<T> io;
    io.r = V.r + base;
    io.v = V.v + base;
    constexpr bool on_s = MODE == MODE_S || MODE == MODE_IN_S;
    io.pz = (on_s ? V.s : V.p) + base;
    io.out = (on_s ? V.sh : V.ph) + base;
    io.c1 = c1;
    io.c2 = c2;
    chain_solve<T, MODE>(pc, pc.block_of[js_[0]], op.nr, io, js_, nk_, lds_of<T>(sh).chain);
  }
}

// BiCGSTAB on A y = rhs for every live instance; y holds the initial guess, r = rhs - A y and
// r^ = r are already written and their partials (SLOT_RHO, SLOT_RR, SLOT_BB) stored; the
// unfinished-work-group counter *cnt already counts this work-group. verify: confirm convergence
// with the true residual (restart on failure). On its final transition an instance writes its
// iterate to dst (when not null, and not when the next step in the launch was prepared from it) and
// its statistics to *so (when not null). The loop ends at the
// first barrier after which no work-group of the launch is unfinished. need_init (when not null):
// counter of instances whose next step in the launch must form its own initial data, incremented
// on the final transition. skip_first: the caller has just passed a grid barrier after which every
// input of the first window is in place (the first window then starts without one).
template <typename T, bool PREC>
__device__ inline void krylov(const SolveArgs& a, const WgInfo& wi, const KVec<T>& V, const c2_t<T>* rhs, size_t base,
                              double tol, int max_iter, bool verify, int* cnt, Inst& st, Shared& sh, Marks& mk,
                              GridBar& gb, c2_t<T>* dst, StatsDev* so, c2_t<T>* bnext_buf, bool from_next,
                              int* need_init = nullptr, bool skip_first = false, c2_t<T>* xalt_buf = nullptr) {
  const double2 ah = make_double2(0.0, 0.5 * a.dt);
  const c2_t<T> ahc = to_c<T>(ah);
  constexpr bool prec = PREC;
  constexpr int kGB = kGatherBatch;
  constexpr int kTR = PREC ? 4 : 2;  // the preconditioned variant has 512 registers per lane
  // the iterate and the other iterate buffer (xalt_buf: x + alpha p^ is formed there with s when the
  // half step may end the solve, and the two buffers swap roles when it does)
  c2_t<T>* x = (st.xsel ? xalt_buf : V.x) + base;
  c2_t<T>* xo = xalt_buf != nullptr ? (st.xsel ? V.x : xalt_buf) + base : nullptr;
  c2_t<T>* r = V.r + base;
  c2_t<T>* rh = V.rh + base;
  c2_t<T>* p = V.p + base;
  c2_t<T>* ph = V.ph + base;
  c2_t<T>* v = V.v + base;
  c2_t<T>* s = V.s + base;
  c2_t<T>* shv = V.sh + base;
  c2_t<T>* t = V.t + base;
  const c2_t<T>* b_ = rhs + base;
  c2_t<T>* bnext = bnext_buf != nullptr ? bnext_buf + base : nullptr;

  // final transition: write back, report, leave the unfinished count (zero_x: the next step starts
  // from a zero guess)
  // A step whose successor in the launch already has its initial data (next_ready) skips the
  // write-back: the successor does not read dst, and writes its own result there.
  auto finish = [&](int state, bool zero_x = false) {
    st.state = state;
    const bool write = dst != nullptr && !(state == ST_DONE && st.next_ready);
    if (write || zero_x)
      elem_own<T>(a, wi, [&](long e) {
        if (write) dst[e] = x[e];
        if (zero_x) x[e] = cmk<T>(0, 0);
      });
    if (need_init != nullptr && !st.next_ready && wi.g == 0 && threadIdx.x == 0)
      __hip_atomic_fetch_add(need_init, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (so != nullptr && wi.g == 0 && threadIdx.x == 0) {
      so->status = status_of(state);
      so->iters = st.iters;
      so->matvecs = st.matvecs;
      so->restarts = st.restarts;
      so->outer_iters = 0;
      so->precs = st.precs;
      so->rel_res = st.rel_res;
      so->true_rel_res = st.true_rel_res;
    }
    counter_add(cnt, -1);
  };
  // converged on the recursive residual
  auto converged = [&]() {
    if (verify) {
      st.state = ST_VERIFY;
    } else {
      st.true_rel_res = st.rel_res;
      finish(ST_DONE);
    }
  };
  // true residual of this step (its norm) together with the next step's right-hand side
  // b' = (S - i dt/2 H') x, residual r' = b' - A' x0 and r^' = r' (H': next step's fields)
  auto fused_check = [&]() {
    double2 acc = make_double2(0.0, 0.0), accb = make_double2(0.0, 0.0), accr = make_double2(0.0, 0.0);
    const c2_t<T> mahc = cmk<T>(-ahc.x, -ahc.y), mdt = cmk<T>(0, (T)(-a.dt));
    const bool prev = a.guess == GUESS_PREV;
    apply_own2<T, kGB, kTR>(a, wi, x, sh, [&](long e, c2_t<T> sx, c2_t<T> hx, c2_t<T> hx2) {
      const c2_t<T> rt = csub<T>(b_[e], cfma<T>(ahc, hx, sx));
      dot_acc(acc, rt, rt);
      const c2_t<T> bn = cfma<T>(mahc, hx2, sx);
      bnext[e] = bn;
      dot_acc(accb, bn, bn);
      const c2_t<T> rn = prev ? cmul<T>(mdt, hx2) : bn;  // x0 = x: b' - A' x = -i dt H' x
      r[e] = rn;
      rh[e] = rn;
      dot_acc(accr, rn, rn);
    });
    put_partial(a, wi, SLOT_RR, acc, sh);
    put_partial(a, wi, SLOT_NBB, accb, sh);
    put_partial(a, wi, SLOT_NRHO, accr, sh);
    put_partial(a, wi, SLOT_NRR, accr, sh);
    st.fused = 1;
  };
  // true-residual states, handled in whichever window comes next (s0: state at window entry)
  auto verify_step = [&](int s0) {
    if (s0 == ST_VERIFY) {
      if (bnext != nullptr && !st.nofuse) {
        fused_check();
      } else {
        double2 acc = make_double2(0.0, 0.0);
        apply_own<T, kGB, kTR>(a, wi, x, sh, [&](long e, c2_t<T> sx, c2_t<T> hx) {
          const c2_t<T> rr = csub<T>(b_[e], cfma<T>(ahc, hx, sx));
          r[e] = rr;
          dot_acc(acc, rr, rr);
        });
        put_partial(a, wi, SLOT_RR, acc, sh);
        put_partial(a, wi, SLOT_AUX, acc, sh);
        st.fused = 0;
      }
      st.matvecs++;
      st.state = ST_VCHECK;
    } else if (s0 == ST_VCHECK) {
      const double rr = get_total(a, wi, SLOT_RR, sh).x;
      st.true_rel_res = st.bb > 0 ? sqrt(rr / st.bb) : 0.0;
      if (rr <= st.target2) {
        st.next_ready = st.fused;
        finish(ST_DONE, st.fused && a.guess == GUESS_ZERO);
      } else if (st.iters >= max_iter) {
        finish(ST_FAILED);
      } else if (st.fused) {
        st.nofuse = 1;  // r now holds the next step's residual: form this step's again, then restart
        st.state = ST_VERIFY;
      } else {
        st.state = ST_PENDING;  // true residual too large: restart from it (AUX holds ||r||^2)
        st.restarts++;
        elem_own<T>(a, wi, [&](long e) { rh[e] = r[e]; });
      }
    }
  };

  while (true) {
    int left = 0;  // work-groups of the launch still unfinished after the barrier
    // ---------------- W0
    if (!skip_first) {
      if (!grid_barrier(gb, cnt, &left)) return;
      if (left == 0) break;
    }
    skip_first = false;
    mk.mark(10);
    int s0 = wi.live ? st.state : ST_INACTIVE;
    bool work = false;
    double2 beta = make_double2(0.0, 0.0);
    if (s0 == ST_ACTIVE || s0 == ST_PENDING) {
      const bool pend = s0 == ST_PENDING;
      const bool nx = st.first && from_next;  // initial partials formed by the previous step
      double2 rho, rrt, bbt;
      get_totals3(a, wi, pend ? SLOT_AUX : (nx ? SLOT_NRHO : SLOT_RHO), nx ? SLOT_NRR : SLOT_RR,
                  nx ? SLOT_NBB : SLOT_BB, rho, rrt, bbt, sh);
      const double rr = pend ? rho.x : rrt.x;
      if (st.first) {
        st.bb = bbt.x;
        st.target2 = tol * tol * st.bb;
        st.first = 0;
      }
      st.rel_res = st.bb > 0 ? sqrt(rr / st.bb) : 0.0;
      if (pend) { st.state = ST_ACTIVE; st.fresh = 1; }
      const double rn = sqrt(rho.x * rho.x + rho.y * rho.y);
      if (!isfinite(rr) || !isfinite(st.bb) || !isfinite(rn)) {
        // a NaN or Inf in the right-hand side, the guess or the iteration: stop at once (the
        // reductions are deterministic, so every work-group of the instance takes this branch)
        st.true_rel_res = st.rel_res;
        finish(ST_NONFINITE);
      } else if (rr <= st.target2) {
        converged();
      } else if (st.iters >= max_iter) {
        finish(ST_FAILED);
      } else {
        const double om = sqrt(st.omega.x * st.omega.x + st.omega.y * st.omega.y);
        // rho = <r^, r> vanishing (also at the start of a cycle, where r^ may be a given shadow
        // residual) or omega vanishing: restart with r^ = r
        if (rn <= 1e-300 * (1.0 + rr) || (!st.fresh && om == 0.0)) {
          // breakdown: restart from the same r with r^ = r; rho of the restart is ||r||^2
          st.restarts++;
          if (st.restarts > 20) {
            finish(ST_BREAKDOWN);
          } else {
            st.state = ST_PENDING;
            double2 acc = make_double2(0.0, 0.0);
            elem_own<T>(a, wi, [&](long e) { rh[e] = r[e]; dot_acc(acc, r[e], r[e]); });
            put_partial(a, wi, SLOT_AUX, acc, sh);
          }
        } else {
          if (!st.fresh) beta = dmul(cdiv(rho, st.rho), cdiv(st.alpha, st.omega));
          st.rho = rho;
          work = true;
        }
      }
    }
    if (work) {
      if constexpr (PREC) {
        if (st.fresh) chains_own<T, MODE_FRESH>(a, wi, V, base, beta, st.omega, sh);
        else chains_own<T, MODE_P>(a, wi, V, base, beta, st.omega, sh);
        st.precs++;
      } else {
        const c2_t<T> bc = to_c<T>(beta), oc = to_c<T>(st.omega);
        const bool fr = st.fresh;
        elem_own<T>(a, wi, [&](long e) {
          p[e] = fr ? r[e] : cfma<T>(bc, csub<T>(p[e], cmul<T>(oc, v[e])), r[e]);
        });
      }
      st.fresh = 0;
    }
    verify_step(s0);
    // ---------------- W1: v = A p^, <r^, v>
    if (!grid_barrier(gb, cnt, &left)) return;
    if (left == 0) break;
    mk.mark(11);
    s0 = wi.live ? st.state : ST_INACTIVE;
    if (s0 == ST_ACTIVE) {
      double2 acc = make_double2(0.0, 0.0);
      apply_own<T, kGB, kTR>(a, wi, prec ? ph : p, sh, [&](long e, c2_t<T> sx, c2_t<T> hx) {
        const c2_t<T> vv = cfma<T>(ahc, hx, sx);
        v[e] = vv;
        dot_acc(acc, rh[e], vv);
      });
      put_partial(a, wi, SLOT_RV, acc, sh);
      st.matvecs++;
    }
    verify_step(s0);
    // ---------------- W2: alpha, s = r - alpha v, ||s||^2
    if (!grid_barrier(gb, cnt, &left)) return;
    if (left == 0) break;
    mk.mark(12);
    s0 = wi.live ? st.state : ST_INACTIVE;
    if (s0 == ST_ACTIVE) {
      const double2 rv = get_total(a, wi, SLOT_RV, sh);
      if (rv.x == 0.0 && rv.y == 0.0) {
        st.state = ST_PENDING;  // breakdown: restart at the next W0 from the same r
        st.restarts++;
        double2 acc = make_double2(0.0, 0.0);
        elem_own<T>(a, wi, [&](long e) { rh[e] = r[e]; dot_acc(acc, r[e], r[e]); });
        put_partial(a, wi, SLOT_AUX, acc, sh);
      } else {
        st.alpha = cdiv(st.rho, rv);
        // the preconditioned s^ is formed only if the half step does not already converge (W3);
        // in the iteration whose half step ended the previous step's solve, when the residual
        // check would also form the next step's data, x + alpha p^ is formed here too, so that the
        // check can run in the window of the test
        double n2 = 0.0;
        const c2_t<T> al = to_c<T>(st.alpha);
        const c2_t<T>* dir = prec ? ph : p;
        const bool ahead = xo != nullptr && verify && bnext != nullptr && !st.nofuse && st.iters == st.spec_it;
        elem_own<T>(a, wi, [&](long e) {
          const c2_t<T> sv = csub<T>(r[e], cmul<T>(al, v[e]));
          s[e] = sv;
          n2 += (double)sv.x * sv.x + (double)sv.y * sv.y;
          if (ahead) xo[e] = cfma<T>(al, dir[e], x[e]);
        });
        st.xahead = ahead;
        put_partial(a, wi, SLOT_SS, make_double2(n2, 0.0), sh);
      }
    }
    verify_step(s0);
    // ---------------- W3: half-step test; s^ = M^-1 s (preconditioned) or t = A s
    if (!grid_barrier(gb, cnt, &left)) return;
    if (left == 0) break;
    mk.mark(13);
    s0 = wi.live ? st.state : ST_INACTIVE;
    if (s0 == ST_ACTIVE) {
      const double ss = get_total(a, wi, SLOT_SS, sh).x;
      if (ss <= st.target2) {
        st.iters++;
        st.rel_res = st.bb > 0 ? sqrt(ss / st.bb) : 0.0;
        if (st.xahead) {
          // x + alpha p^ is in the other buffer: it becomes the iterate, and its residual check
          // (with the next step's initial data) runs in this window
          c2_t<T>* tmp = x;
          x = xo;
          xo = tmp;
          st.xsel ^= 1;
          fused_check();
          st.matvecs++;
          st.state = ST_VCHECK;
        } else {
          const c2_t<T> al = to_c<T>(st.alpha);
          const c2_t<T>* dir = prec ? ph : p;
          elem_own<T>(a, wi, [&](long e) { x[e] = cfma<T>(al, dir[e], x[e]); });
          converged();
        }
      } else if constexpr (PREC) {
        chains_own<T, MODE_IN_S>(a, wi, V, base, st.alpha, st.alpha, sh);  // s^ = K^-1 s
        st.precs++;
      } else {
        double2 ts = make_double2(0.0, 0.0), tt = make_double2(0.0, 0.0);
        apply_own<T, kGB, kTR>(a, wi, s, sh, [&](long e, c2_t<T> sx, c2_t<T> hx) {
          const c2_t<T> tv = cfma<T>(ahc, hx, sx);
          t[e] = tv;
          dot_acc(ts, tv, s[e]);
          dot_acc(tt, tv, tv);
        });
        put_partial(a, wi, SLOT_TS, ts, sh);
        put_partial(a, wi, SLOT_TT, tt, sh);
        st.matvecs++;
      }
    }
    verify_step(s0);
    if constexpr (PREC) {
      // ---------------- W3b: t = A s^
      if (!grid_barrier(gb, cnt, &left)) return;
      if (left == 0) break;
      mk.mark(15);
      s0 = wi.live ? st.state : ST_INACTIVE;
      if (s0 == ST_ACTIVE) {
        double2 ts = make_double2(0.0, 0.0), tt = make_double2(0.0, 0.0);
        apply_own<T, kGB, kTR>(a, wi, shv, sh, [&](long e, c2_t<T> sx, c2_t<T> hx) {
          const c2_t<T> tv = cfma<T>(ahc, hx, sx);
          t[e] = tv;
          dot_acc(ts, tv, s[e]);
          dot_acc(tt, tv, tv);
        });
        put_partial(a, wi, SLOT_TS, ts, sh);
        put_partial(a, wi, SLOT_TT, tt, sh);
        st.matvecs++;
      }
      verify_step(s0);
    }
    // ---------------- W4: omega, x, r, <r^, r>, ||r||^2
    if (!grid_barrier(gb, cnt, &left)) return;
    if (left == 0) break;
    mk.mark(14);
    s0 = wi.live ? st.state : ST_INACTIVE;
    if (s0 == ST_ACTIVE) {
      double2 ts, ttt, unused;
      get_totals3(a, wi, SLOT_TS, SLOT_TT, SLOT_TT, ts, ttt, unused, sh);
      const double tt = ttt.x;
      st.omega = tt > 0.0 ? make_double2(ts.x / tt, ts.y / tt) : make_double2(0.0, 0.0);
      const c2_t<T> al = to_c<T>(st.alpha), om = to_c<T>(st.omega);
      const c2_t<T>* pd = prec ? ph : p;
      const c2_t<T>* sd = prec ? shv : s;
      double2 rho = make_double2(0.0, 0.0), rr = make_double2(0.0, 0.0);
      elem_own<T>(a, wi, [&](long e) {
        x[e] = cfma<T>(om, sd[e], cfma<T>(al, pd[e], x[e]));
        const c2_t<T> rv = csub<T>(s[e], cmul<T>(om, t[e]));
        r[e] = rv;
        dot_acc(rho, rh[e], rv);
        dot_acc(rr, rv, rv);
      });
      put_partial(a, wi, SLOT_RHO, rho, sh);
      put_partial(a, wi, SLOT_RR, rr, sh);
      st.iters++;
    }
    verify_step(s0);
  }
}

// Per-thread constants of the calling thread's coupling term m = threadIdx.x for its instance:
// prefactor, and either the pulse (time steps) or the explicit field value (single solves).
struct TermRegs {
  double2 coef;
  PulseDev pulse;
  double fval;
  int fi;  // field index of the term
};

__device__ inline TermRegs term_regs(const SolveArgs& a, const WgInfo& wi) {
  TermRegs tr{};
  const int m = threadIdx.x;
  if (m < a.op64.n_terms && wi.live) {
    tr.coef = a.op64.t_coef[m];
    const int fi = a.op64.t_field[m];
    tr.fi = fi;
    if (a.mode == MODE_STEP) tr.pulse = a.pulses[(size_t)wi.b * a.n_fields + fi];
    else tr.fval = a.fvals[(size_t)wi.b * a.n_fields + fi];
  }
  return tr;
}

// Field values of step `step` (time steps: row `step` of the field table, or the pulses at its
// midpoint; single solves: the explicit values) into the term table (live: the instance takes part;
// else all zero).
__device__ inline void fields_to_lds(const SolveArgs& a, const TermRegs& tr, const WgInfo& wi, bool live, int step,
                                     TermLds& tl) {
  terms_fields(a.op64.n_terms, a.op64.n_groups, tl, [&](int) {
    if (!live) return make_double2(0.0, 0.0);
    double f = tr.fval;
    if (a.mode == MODE_STEP)
      f = a.ftab != nullptr ? a.ftab[((size_t)wi.b * a.ftab_rows + step) * a.n_fields + tr.fi]
                            : pulse_eval(tr.pulse, mid_time(a.t0, step, a.dt));
    return make_double2(tr.coef.x * f, tr.coef.y * f);
  });
}

// After a grid-barrier time-out: report the unfinished steps of the instance as failed launches.
__device__ inline void fail_steps(const SolveArgs& a, const WgInfo& wi, int k) {
  if (a.stats == nullptr || !wi.live || wi.g != 0 || threadIdx.x != 0) return;
  for (int kk = k; kk < a.n_chunk; ++kk) {
    StatsDev& o = a.stats[(size_t)kk * a.B + wi.b];
    o.status = -2;  // TDDE_ERR_HIP
    o.iters = o.matvecs = o.restarts = o.outer_iters = o.precs = 0;
    o.rel_res = o.true_rel_res = 0.0;
  }
}

template <bool PREC, bool MIXED>
__global__ __attribute__((amdgpu_flat_work_group_size(kThreads, kThreads), amdgpu_waves_per_eu(PREC ? 1 : 2)))
void persistent_kernel(SolveArgs a) {
  __shared__ Shared sh;
  Marks mk{a.marks, 0, a.n_marks};
  GridBar gb{a.bar, (unsigned)a.n_wg, 0u, false};
  WgInfo wi;
  wi.G = a.G;
  wi.live = blockIdx.x < (unsigned)(a.B * a.G);
  wi.b = wi.live ? blockIdx.x / a.G : 0;
  wi.g = wi.live ? blockIdx.x % a.G : 0;
  const size_t base = (size_t)wi.b * a.E;
  const double2 ah = make_double2(0.0, 0.5 * a.dt);
  const c2_t<double> ahc = ah, mahc = make_double2(0.0, -0.5 * a.dt);

  // term tables: group layout once per launch, field values per step
  terms_layout<double>(a.op64, sh.tl);
  terms_layout<double>(a.op64, sh.tl2);
  const TermRegs treg = term_regs(a, wi);
  bool ready = false;  // this step's b, x0, r, r^ and partials were formed by the previous step
  int xsel = 0;        // the iterate of a ready step lives in the second iterate buffer
  int spec_it = 0;     // the previous step's last iteration (its half step is tested ahead)
  for (int k = 0; k < a.n_chunk; ++k) {
    const int step = a.step0 + k;
    int* cnt = a.counters + (size_t)k * kCounterPerStep;
    // the FP64 solve of the previous step ended at a grid barrier after its last write
    if (MIXED && k > 0 && !grid_barrier(gb)) { fail_steps(a, wi, k); return; }
    mk.mark(1);
    const bool inst = wi.live && (a.mode == MODE_SOLVE || a.n_steps == nullptr || step < a.n_steps[wi.b]);
    WgInfo wk = wi;
    wk.live = inst;
    fields_to_lds(a, treg, wi, inst, step, sh.tl);
    // the residual check of this step also forms the next step's right-hand side when the next
    // step runs in this launch for this instance
    const bool next_live = wi.live && k + 1 < a.n_chunk && (a.n_steps == nullptr || step + 1 < a.n_steps[wi.b]);
    const bool fuse = !MIXED && a.mode == MODE_STEP && a.guess != GUESS_GIVEN && inst && next_live;
    if (!MIXED && a.mode == MODE_STEP && a.guess != GUESS_GIVEN) fields_to_lds(a, treg, wi, fuse, step + 1, sh.tl2);
    if (!inst) ready = false;
    // right-hand side buffers alternate between steps so the next one can be formed early
    double2* bbuf = (!MIXED && (k & 1)) ? a.bvec2 : a.bvec;
    double2* bnbuf = (k & 1) ? a.bvec : a.bvec2;

    Inst st = {};
    st.state = inst ? ST_ACTIVE : ST_INACTIVE;
    st.fresh = 1;
    st.first = 1;
    st.xsel = ready ? xsel : 0;
    st.spec_it = spec_it;
    st.omega = make_double2(1.0, 0.0);
    st.alpha = make_double2(1.0, 0.0);
    st.rho = make_double2(1.0, 0.0);

    KVec<double> V = a.v64;
    double2* x = V.x + base;
    double2* bv = bbuf + base;
    // ---- right-hand side b = (S - i dt/2 H) psi and the initial guess
    if (inst && !ready) {
      if (a.mode == MODE_STEP) {
        double2 bb = {0, 0}, rr = {0, 0};
        const double2* psi = a.psi + base;
        const int gs = a.guess;
        const bool direct_r = !MIXED && gs != GUESS_GIVEN;
        apply_own<double, kGatherBatch, PREC ? 4 : 2>(a, wk, psi, sh, [&](long e, double2 sx, double2 hx) {
          const double2 bval = cfma<double>(mahc, hx, sx);
          bv[e] = bval;
          dot_acc(bb, bval, bval);
          if (gs == GUESS_PREV) x[e] = psi[e];
          else if (gs == GUESS_ZERO) x[e] = make_double2(0.0, 0.0);
          else x[e] = a.guess_in[base + e];
          if (direct_r) {
            // r = b - A x0: for x0 = psi it is -i dt H psi; for x0 = 0 it is b
            const double2 rv = gs == GUESS_PREV ? cmul<double>(make_double2(0.0, -a.dt), hx) : bval;
            V.r[base + e] = rv;
            V.rh[base + e] = rv;
            dot_acc(rr, rv, rv);
          }
        });
        put_partial(a, wk, MIXED ? SLOT_OBB : SLOT_BB, bb, sh);
        if (direct_r) { put_partial(a, wk, SLOT_RHO, rr, sh); put_partial(a, wk, SLOT_RR, rr, sh); }
        st.matvecs++;
      } else {
        // MODE_SOLVE: copy b and the guess into the workspace
        double2 bb = {0, 0};
        elem_own<double>(a, wk, [&](long e) {
          const double2 bval = a.b_in[base + e];
          bv[e] = bval;
          dot_acc(bb, bval, bval);
          x[e] = a.guess == GUESS_ZERO ? make_double2(0.0, 0.0) : a.x_io[base + e];
        });
        put_partial(a, wk, MIXED ? SLOT_OBB : SLOT_BB, bb, sh);
      }
    }
    const bool need_r = MIXED || a.guess == GUESS_GIVEN || a.mode == MODE_SOLVE;
    if (need_r) {
      // r = b - A x0 in FP64 (the outer residual in mixed precision)
      if (!grid_barrier(gb)) { fail_steps(a, wi, k); return; }
      if (inst) {
        double2 rr = {0, 0}, rho = {0, 0};
        double2* rt = MIXED ? a.r64 + base : V.r + base;
        const double2* shadow = !MIXED && a.shadow != nullptr ? a.shadow + base : nullptr;
        apply_own<double, kGatherBatch, PREC ? 4 : 2>(a, wk, x, sh, [&](long e, double2 sx, double2 hx) {
          const double2 rv = csub<double>(bv[e], cfma<double>(ahc, hx, sx));
          rt[e] = rv;
          if (!MIXED) {
            // shadow residual of the first cycle: r^ = r, or the caller's vector (test hook)
            const double2 rhv = shadow != nullptr ? shadow[e] : rv;
            V.rh[base + e] = rhv;
            dot_acc(rho, rhv, rv);
          }
          dot_acc(rr, rv, rv);
        });
        if (!MIXED) {
          put_partial(a, wk, SLOT_RHO, rho, sh);
          put_partial(a, wk, SLOT_RR, rr, sh);
        } else {
          put_partial(a, wk, SLOT_ORR, rr, sh);
        }
        st.matvecs++;
      }
    }

    if constexpr (!MIXED) {
      if (inst) counter_add(cnt, 1);
      double2* dst = (a.mode == MODE_STEP ? a.psi : a.x_io) + base;
      StatsDev* so = a.stats != nullptr ? a.stats + (size_t)k * a.B + wk.b : nullptr;
      // Steps after the first: the previous step's solve ended at a grid barrier, and when no
      // instance has to form its own initial data (count of the previous step's final transitions
      // without the next step's data in place, complete at that barrier) nothing has been written
      // since, so the first window needs no barrier of its own. The count is the same in every
      // work-group, so every work-group makes the same choice.
      const bool chained = a.mode == MODE_STEP && a.guess != GUESS_GIVEN;
      const bool skip = chained && k > 0 &&
                        __hip_atomic_load(a.counters + (size_t)k * kCounterPerStep + 1, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT) == 0;
      int* need_next = chained && k + 1 < a.n_chunk ? a.counters + (size_t)(k + 1) * kCounterPerStep + 1 : nullptr;
      krylov<double, PREC>(a, wk, V, bbuf, base, a.tol, a.max_iter, true, cnt, st, sh, mk, gb, dst, so,
                           fuse ? bnbuf : nullptr, ready, need_next, skip, a.xalt);
      ready = inst && st.next_ready;
      xsel = st.xsel;
      spec_it = st.iters > 0 ? st.iters - 1 : 0;
      if (gb.failed) { fail_steps(a, wi, k); return; }
    } else {
      // ---- FP64 iterative refinement around an FP32 BiCGSTAB (inner residuals, dots in FP64)
      KVec<float> U = a.v32;
      int outer_state = inst ? ST_ACTIVE : ST_INACTIVE;
      int total_iters = 0, total_mv = st.matvecs, outer = 0, total_precs = 0;
      double bb = 0.0;
      int* ocnt = cnt + 1;
      if (inst) counter_add(ocnt, 1);
      for (int it = 0;; ++it) {
        if (!grid_barrier(gb)) { fail_steps(a, wi, k); return; }
        int* icnt = cnt + 2 + (it % (kCounterPerStep - 2));
        Inst ist = {};
        ist.state = ST_INACTIVE;
        double rnorm = 0.0;
        if (outer_state == ST_ACTIVE) {
          const double rr = get_total(a, wk, SLOT_ORR, sh).x;
          if (it == 0) bb = get_total(a, wk, SLOT_OBB, sh).x;
          st.rel_res = st.true_rel_res = bb > 0 ? sqrt(rr / bb) : 0.0;
          if (rr <= a.tol * a.tol * bb) {
            outer_state = ST_DONE;
            counter_add(ocnt, -1);
          } else if (it >= a.max_outer) {
            outer_state = ST_FAILED;
            counter_add(ocnt, -1);
          } else {
            rnorm = sqrt(rr);
            const double sc = 1.0 / rnorm;
            const double2* r64 = a.r64 + base;
            double2 rho = {0, 0};
            elem_own<float>(a, wk, [&](long e) {
              const float2 z = make_float2((float)(r64[e].x * sc), (float)(r64[e].y * sc));
              a.rhs32[base + e] = z;
              U.r[base + e] = z;
              U.rh[base + e] = z;
              U.x[base + e] = make_float2(0.f, 0.f);
              dot_acc(rho, z, z);
            });
            put_partial(a, wk, SLOT_RHO, rho, sh);
            put_partial(a, wk, SLOT_RR, rho, sh);
            put_partial(a, wk, SLOT_BB, rho, sh);
            ist.state = ST_ACTIVE;
            ist.fresh = 1;
            ist.first = 1;
            ist.omega = ist.alpha = ist.rho = make_double2(1.0, 0.0);
            counter_add(icnt, 1);
            outer++;
          }
        }
        if (!grid_barrier(gb)) { fail_steps(a, wi, k); return; }
        if (__hip_atomic_load(ocnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) break;
        WgInfo wq = wk;
        wq.live = ist.state == ST_ACTIVE;
        krylov<float, PREC>(a, wq, U, a.rhs32, base, a.inner_tol, a.max_iter, false, icnt, ist, sh, mk, gb, nullptr,
                            nullptr, nullptr, false);
        total_iters += ist.iters;
        total_mv += ist.matvecs;
        total_precs += ist.precs;
        // x += ||r|| d (FP64), then r = b - A x (FP64)
        if (!grid_barrier(gb)) { fail_steps(a, wi, k); return; }
        if (wq.live) {
          const float2* d = U.x + base;
          elem_own<double>(a, wk, [&](long e) {
            x[e].x += rnorm * (double)d[e].x;
            x[e].y += rnorm * (double)d[e].y;
          });
        }
        if (!grid_barrier(gb)) { fail_steps(a, wi, k); return; }
        if (wq.live) {
          double2 rr = {0, 0};
          double2* rt = a.r64 + base;
          apply_own<double, kGatherBatch, PREC ? 4 : 2>(a, wk, x, sh, [&](long e, double2 sx, double2 hx) {
            const double2 rv = csub<double>(bv[e], cfma<double>(ahc, hx, sx));
            rt[e] = rv;
            dot_acc(rr, rv, rv);
          });
          put_partial(a, wk, SLOT_ORR, rr, sh);
          total_mv++;
        }
      }
      st.iters = total_iters;
      st.matvecs = total_mv;
      st.state = outer_state == ST_DONE ? ST_DONE : (outer_state == ST_INACTIVE ? ST_INACTIVE : ST_FAILED);
      st.restarts = outer;  // reported as outer iterations below

      // ---- write back and statistics (the FP64 path does both as each instance finishes)
      if (!grid_barrier(gb)) { fail_steps(a, wi, k); return; }
      mk.mark(2);
      if (inst) {
        double2* dst = a.mode == MODE_STEP ? a.psi + base : a.x_io + base;
        elem_own<double>(a, wk, [&](long e) { dst[e] = x[e]; });
        if (a.stats != nullptr && wk.g == 0 && threadIdx.x == 0) {
          StatsDev& o = a.stats[(size_t)k * a.B + wk.b];
          o.status = status_of(st.state);
          o.iters = st.iters;
          o.matvecs = st.matvecs;
          o.restarts = 0;
          o.outer_iters = st.restarts;
          o.precs = total_precs;
          o.rel_res = st.rel_res;
          o.true_rel_res = st.true_rel_res;
        }
      }
    }
  }
  grid_barrier(gb);
  mk.mark(3);
}

}  // namespace tdde
