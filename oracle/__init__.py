"""CPU oracle for Discrete Iterative Filtering and its FFT direct form.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import anything from this package.  The
GPU library under ``paper_1802_01359_amd/`` shares no code with it and never
imports it.

- ``dif``: plain FP64 time-domain iteration of Algorithm 2 (C, built with gcc);
- ``fif_spectral``: the paper's Section 4 direct form in FP64 with numpy's FFT,
  scanning N0 = 1, 2, ... until SD <= delta.

Every function here is pinned by ``tests/test_oracle_*.py`` against closed
forms, invariants and brute force on tiny inputs.
"""
