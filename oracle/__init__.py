"""Plain FP64 CPU oracle for the event-parallel matrix-element hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or execute anything in this package; only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the GPU path.

The paper (Carrazza, Cruz-Martinez, Palazzo, "Extending MadFlow:
device-specific optimization", ICHEP 2022) describes event-axis parallel Monte
Carlo (abstract; sect. 1), Vegas integration (sect. 1) and auto-generated
tree-level matrix elements built from external wavefunctions, vertices and
propagators (sect. 2, Fig. 2) but prints no formulas.  Each module therefore
writes out the textbook definition of the quantity it computes and cites it:

* ``philox``       Philox4x32-10 counter RNG (Salmon et al., SC'11)
* ``kinematics``   Minkowski algebra, boosts
* ``phase_space``  RAMBO on diet (Plaetzer 2013) + massive rescaling
                   (Kleiss, Stirling, Ellis 1986); classic RAMBO for cross-checks
* ``wavefunctions`` HELAS-convention spinors and polarisation vectors
                   (Murayama, Watanabe, Hagiwara, KEK-91-11)
* ``colour``       SU(3) generators, structure constants, colour matrices by
                   brute-force traces
* ``me_explicit``  sum of all tree Feynman diagrams with explicit colour
                   (full QCD Feynman rules, Peskin & Schroeder Fig. 16.7),
                   organised as an off-shell recursion over external-leg subsets
* ``me_ordered``   colour-ordered partial amplitudes + colour matrix
* ``closed_forms`` e+e- -> mu+mu-, LO gg -> ttbar, phase-space volumes, cross sections
* ``cuts``, ``vegas``, ``integrand``, ``grad``
"""
