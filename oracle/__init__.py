"""FP64 CPU oracle for compressed NMF with random projections (FastHALS-RP).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP library (no kernels, headers, helpers, tables or constant generators) and it
never reads a value produced by the HIP path.

Modules
-------
nmf     -- range finder (eq 3.5, Sec 3.1), CholeskyQR2, sketches (Sec 4),
           FastHALS-RP (eq fastHALS_a), plain FastHALS (Sec 2.2), naive
           HALS-RP (eqs 4_6 and hals_update), the sparsity/smoothness rule
           (Sec 4.1), residuals (eq 2.2), Gini coefficient (Sec 5.1).
philox  -- Philox4x32-10 counter-based generator (Salmon et al., SC'11) and the
           Box-Muller transform used for the Gaussian test matrix (Sec 3).
quant   -- BF16 round-to-nearest-even and OCP FP8 e4m3 with 128x128 block
           scales (the low-precision compression extension).
mlp     -- learned warm start: k'->512->512->r MLP, FP64 forward, backward,
           Adam, warm-start selection (extension; the paper is silent on it).

Every function is plain FP64 NumPy, written for checkability, not speed.
"""
