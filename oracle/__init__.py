"""Plain FP64 CPU oracle for the Crank-Nicolson / BiCGSTAB time step.

TEST INFRASTRUCTURE ONLY. Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything here. The GPU
library never uses it and shares no code with it.

Contents (each function cites the passage of the paper it restates):
  * ``fields``     time functions f(t) of the laser pulse (eq. ndpPot, eq. bdpA)
  * ``assemble``   CSR assembly of H0, S, the coupling terms and H(t) (eq. fullH)
  * ``rows``       element-wise definition of y = a_S S x + a_H H x at chosen rows
  * ``bicgstab``   textbook unpreconditioned BiCGSTAB (van der Vorst 1992)
  * ``step``       the Crank-Nicolson step (eq. solPsi, midpoint time of Sec. 2.4)
  * ``mlp``        FP64 forward / backward / Adam of the learned initial-guess network
  * ``spectrum``   photoelectron energy spectrum dP/dE and its error integral (eq. dPdE)

Parity status: every function is pinned by the non-GPU tests (dense solves, closed
forms, invariants, brute force on tiny inputs, finite differences). Iteration counts
of BiCGSTAB are reported, never gated ("parity unpinned": different valid
implementations give different iterates).
"""
