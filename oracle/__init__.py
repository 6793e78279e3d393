"""Plain FP64 CPU oracle for the PODECM reduced-order model.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU product path imports, links or
executes anything in this package; only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may.  The oracle shares no code with the
HIP path: the two meet only through the ROM artifact file (written here by the
offline stage, read by the library's ``rom_load``) and through the seeded input
generators in ``workloads``, which hold none of the method's arithmetic.

Modules follow the paper (Guo, Rokos, Veroy, arXiv 2307.16894):

* ``material``  -- Appendix A: small-strain J2 with linear isotropic hardening
                   lifted to finite strain by the multiplicative split and the
                   logarithmic elastic strain; tangent by complex-step.
* ``mesh``      -- parent-domain T6 meshes, 3-point interior quadrature.
* ``fem``       -- periodic fluctuation space, gradient operator, assembly of
                   the mapped weak form (Sec. 2.1, eq. weakform-dep-mapped).
* ``auxiliary`` -- Sec. 3.4: auxiliary linear-elastic transformation problem.
* ``fom``       -- full-order Newton solve and effective quantities (Sec. 2).
* ``pod``       -- Sec. 3.1 / 3.2 POD of fluctuation and weighted-stress
                   snapshots.
* ``ecm``       -- Sec. 3.2 greedy empirical cubature with NNLS weights.
* ``rom``       -- Sec. 3.2-3.3 hyper-reduced online solve and effective
                   stress / stiffness; Algorithm 1 (online).
* ``artifact``  -- the ROM artifact file format (writer and reader).
* ``build_rom`` -- Algorithm 1 (offline) driver: writes ROM artifacts.

Every floating-point computation is FP64 (complex128 inside the complex-step
tangent).
"""
