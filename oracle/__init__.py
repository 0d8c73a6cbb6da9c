"""FP64 CPU oracle for near-field XL-MIMO Gram, beamforming rates and saturation.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy/SciPy implementation of what the HIP path computes, written from the
paper (Cui, Park, Alouini, "Channel Capacity Saturation Point and Beamforming
Acceleration for Near-Field XL-MIMO Multiuser Communications").  It shares no
code with the HIP library and imports nothing from the product package; the
only common input is ``workloads`` (seeded drops, no method arithmetic).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product path never calls it.

Modules
  geometry    element coordinates of the ULA / UPA (Sec. II-A)
  channel     spherical-wave channel entries, eq. (3) and free space; exact Gram
  closedform  closed-form power eq. (4)-(5), SPM correlation eq. (6)-(8),
              modified-ZF Gram eqs. (22)-(23), and derived free-space / UPA forms
  rates       ZF / MMSE / MRC / capacity eq. (9) / mismatched modified ZF
  saturation  power saturation eqs. (10)-(20) and Appendix B
  mlp         FP64 reference of the learned residual correction (not in the paper)

Parity status of every function is stated in its docstring; functions with no
independent pin say "parity unpinned".
"""
