"""Plain FP64 CPU oracle for the variational deterministic-particle scheme (VDS)
and its POD model-order reduction.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
anything here.  The GPU library never calls into this package, and this package
imports nothing from the GPU library: the two share no code, no tables and no
helpers.  The one shared module is `workloads`, which draws seeded inputs and
holds none of the method's arithmetic.

Every function is the plain definition written out in float64 with direct
differences (no norm expansion, no blocking beyond bounding memory), so that a
reader can check it against the paper by eye.  Module map:

  vds.py   particle scheme: kernel sums, drift, explicit/implicit Euler,
           stress, energy, dissipation (Sections 2.1-2.2, Appendix A)
  pod.py   snapshot matrix, POD basis, projection/reconstruction (Sections 1.3,
           2.3, 3.1)
  rom.py   Galerkin reduced operators and reduced Euler stepper (Section 2.4)
  mlp.py   learned reduced-step model (not in the paper): MLP forward,
           backward, Adam
"""
