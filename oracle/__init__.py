"""FP64 CPU oracle of the LaueOT hot path (Kacprzak et al., Laue Indexing with
Optimal Transport).

This package is TEST INFRASTRUCTURE.  It is a plain, slow, NumPy FP64
restatement of what the paper computes, written from the paper's equations
and algorithms, and it shares no code with the HIP library.  Only the tests,
the smoke check and the benchmark's CPU-baseline leg may import it; the
product path never does.

Modules
  philox     counter-based random numbers (Philox4x32-10, published definition)
  crystal    cubic plane lists (Sec. 3.1), rotations, the cubic point group
  forward    forward model: Eqs ray_mnt, s_mnt, wavelength, model_spot_cut
  simulate   synthetic detected spots with the ray-noise model (Sec. 3.3.1)
  cost       the pairwise likelihood L_ij of Sec. 4 as a chord cost in mm^2
  sinkhorn   entropic OT E-step with outlier row/column (Eqs update_L, estep_obj,
             Alg. BalancedOT), in the log domain
  mstep      per-grain M-step (Eq. mstep_obj): Gauss-Newton over rotation and
             position, plus the paper's position Newton, rotation MM and Wahba
  em         the multigrain Sinkhorn-EM driver (Alg. LaueOT)
  metrics    misorientation reduced over the cubic group, recall

Parity pins for every function live in tests/test_oracle_*.py.
"""
