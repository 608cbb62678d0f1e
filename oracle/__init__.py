"""Plain FP64 CPU oracle for cut-circuit reconstruction (test infrastructure).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call, link
or execute anything in this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library.

Contents (each function cites the passage of Tang et al., "CutQC: Using Small
Quantum Computers for Large Quantum Circuit Evaluations", ASPLOS '21, that it
follows):

  statevector  own FP64 state-vector simulator (ground truth, Section 2)
  variants     subcircuit variants, shot attribution (Eq. 3) and the p_{1,i},
               p_{2,i} term construction (Section 3.2), Pauli and eigen forms
               (Eq. 1, Eq. 2)
  fd           full-definition build by its plain definition (Section 3.2.3,
               Section 3.3: 4^K Kronecker products scaled by 2^-K) and the
               Eq. 14 cost model
  dd           dynamic definition (Algorithm 1, Section 4.3)
  blocked      full FD vectors in bounded memory (2^30 outputs): the same
               definition with each label summed as soon as both of its
               subcircuits are multiplied in (distributivity; the progressive
               build Eq. 14 counts), one output block at a time
  adjoint      gradient of a loss on the reconstructed distribution with
               respect to every entry tensor, by its plain definition, over
               the whole tensor (vjp) or at chosen elements (vjp_at)
  metrics      relative L1, chi^2 (Eq. 16), cancellation factor kappa
  native       C/OpenMP twin of the FD definition, used for CPU timing

Pins: see tests/test_oracle_*.py.  Every function is checked against brute-force
state-vector simulation of the uncut circuit, closed forms, special cases that
reduce to library routines, or invariants; none is "parity unpinned".
"""
