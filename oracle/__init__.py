"""FP64 CPU oracle for the T2-Shuffling subspace PICS solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.
The product path (``paper_1809_04195_amd``) never imports, links or executes
it, and this package imports nothing from the product path.

Contents
--------
``t2s``   centred 2D DFT, forward / adjoint subspace operator, space-time kernel
          Psi, both normal-operator routes, LLR singular-value soft threshold
          (single-pass and explicit forms), SplitMix64 shift schedule, CG, ADMM,
          FISTA and the objective.
``unet``  (if present) the warm-start network's forward / backward in FP64.
"""
