// Kernel-per-window BiCGSTAB for the Crank-Nicolson step (eq. solPsi, right preconditioner of
// eq. matrixM when enabled): the iteration of the persistent solver with every window of it a kernel
// of its own, each launched at the occupancy its own registers allow. The persistent kernel with the
// preconditioner holds one work-group per CU (its chain solve and apply share one register budget),
// which leaves the apply latency-bound on large instances; here the applies and chain solves run two
// work-groups per CU and the vector updates more.
//
// The scalar recurrence (rho, alpha, omega, beta, the convergence tests, restarts and the
// statistics) lives in device memory, one control block per instance. Every kernel reads its
// instance's block when it starts and works only in the states it serves. A kernel that forms dot
// products writes one partial per work-group; the last work-group of the instance to finish (an
// atomic arrival count) sums the partials in work-group order, so the sums are deterministic, and
// takes the next decision. The host enqueues whole iterations (a fixed sequence of kernels) and
// reads, one iteration behind, how many instances are unfinished; kernels enqueued past the end do
// nothing.
//
// Iteration (one "block" of kernels), by control state:
//   prologue  INIT: b = (S - i dt/2 H) psi, r = r^ = b - A psi (initial guess psi), ||b||, ||r||
//             RESTART: r^ = r, ||r||  (rho of the new cycle)
//   dir       ACTIVE: p = r (new cycle) or r + beta (p - omega v); p^ = K^-1 p
//   apply_v   ACTIVE: v = A p^, <r^, v>              -> alpha
//   s         ACTIVE: s = r - alpha v, ||s||          -> half-step test (HALF)
//   chain_s   ACTIVE: s^ = K^-1 s
//   apply_t   ACTIVE: t = A s^, <t, s>, <t, t>        -> omega
//   xr        ACTIVE: x += alpha p^ + omega s^, r = s - omega t, <r^, r>, ||r||  -> beta / tests
//             HALF: x += alpha p^
//   check     HALF, VERIFY: true residual of the step; when the next step of the call follows, also
//             its right-hand side b' = (S - i dt/2 H') x and r' = r^' = b' - A' x (fused)
//             VERIFY_NF: true residual alone
//   sync      unfinished-instance count to host memory
// The iterate x is the caller's state psi itself (the initial guess of a step is the previous state).
#pragma once
#include "common.hpp"
#include "precond.hpp"

namespace tdde {

enum { SP_FINISHED = 0, SP_INIT = 1, SP_ACTIVE = 2, SP_HALF = 3, SP_VERIFY = 4, SP_VERIFY_NF = 5, SP_RESTART = 6 };

// Partial slots of the kernel-per-window solver ([B][G][kSpSlots] complex values).
enum { SPS_A = 0, SPS_B, SPS_C, kSpSlots };

struct SplitCtl {
  int state;
  int step;      // absolute step of the solve in progress
  int k;         // its row in the statistics (step minus the call's first step)
  int iters, matvecs, restarts, precs;
  int fresh;     // the next direction update starts a cycle (p = r)
  int nofuse;    // a fused check failed: form this step's residual alone from now on
  int par;       // right-hand-side buffer of this step (the next step's is formed in the other)
  int pad0, pad1;
  double2 rho, alpha, omega, beta;
  double bb, target2, rel_res, true_rel_res;
};

constexpr int kSpCntLine = 64;  // ints per arrival counter (one 256-byte line per instance)

struct SplitArgs {
  DevOp<double> op;
  DevPrec<double> pc;
  DevPrec<float> pc32;     // the same factors rounded to FP32 (used when prec32 is set)
  double2 *x, *r, *rh, *p, *ph, *v, *s, *sh, *t;  // ph == p, sh == s without the preconditioner
  double2* bvec[2];        // right-hand sides of this step and the next
  double2* part;           // [B][G][kSpSlots]
  SplitCtl* ctl;           // [B]
  int* cnt;                // [B][kSpCntLine] arrival counters, zero between kernels
  void* stats;             // [n_chunk][B] statistics rows (tdde_solve_stats layout) or null
  const int* n_steps;      // [B]
  const PulseDev* pulses;   // [B][n_fields]
  const double* ftab;      // [B][ftab_rows][n_fields] field table, or null (the pulses)
  int* host_flag;          // host-visible [2]: unfinished instances after a block, by block parity
  int ftab_rows, n_fields;
  int B, E, G;             // G: work-groups per instance of the apply and vector kernels (multiple of 8)
  int step0, n_chunk, max_iter, use_prec, prec32;
  double tol, dt, t0;
};

// Launch one block (one iteration of every unfinished instance) on the stream; parity: block index
// mod 2 (the host-flag slot its sync kernel writes). first: launch the kernel that initialises the
// control blocks before it.
// ev_v: when not null, events recorded right before and after the apply kernel v = A p^.
hipError_t split_launch_block(const SplitArgs& a, hipStream_t stream, int parity, bool first,
                              const hipEvent_t* ev_v = nullptr);

}  // namespace tdde
