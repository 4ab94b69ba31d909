"""Plain FP64 CPU oracle for the selected density matrix (TEST INFRASTRUCTURE ONLY).

This package is the slow, obviously-correct reference that the GPU library is
checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import it.  The product library never calls
into it, and it shares no code with the product: it reads the same seeded
inputs (from ``synth``) and nothing else.

Modules
  poles   -- continued-fraction poles z_p and residues R_p of the Fermi
             function (paper Sec. II B, Eq. (7)), plus an independent
             backward-recurrence evaluation of the truncated fraction.
  dense   -- dense generalized eigenproblem H c = eps S c (Eq. (2)), Fermi
             occupations, rho on the pattern (Eq. (5) / Lehmann form Eq. (9)),
             the per-pole dense inverse and pole sum (Eqs. (6), (8)), S^{-1}
             and the half-filling chemical potential.
  chain   -- closed forms for open tight-binding chains (no eigensolver).
  sampled -- sampled-column reference for systems too large for dense
             algebra (iterative solves of (alpha_p S - H) x = e_j).
"""
