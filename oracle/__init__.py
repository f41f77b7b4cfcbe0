"""Plain FP64 CPU oracle for the CTMRG hot path of TeNeS (arXiv:2112.13184).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: it exists so that ``tests/``, the smoke check and the
CPU-baseline leg of the benchmark can check the GPU library against a slow,
obviously correct implementation.  It shares no code with the GPU path.

Modules
-------
philox        Philox4x64-10 counter-based generator and the sketch matrix
              used by the randomized SVD (Sec. 2.2, partial SVD).
ctmrg         environment, enlarged corners, projectors, directional moves
              and sweeps (Sec. 2.2, Fig. 2).
observables   reduced density matrices, expectation values, ln(kappa),
              impurity ratios, correlation functions (Sec. 5.3, Eq. (8)).
closed_forms  Onsager / Yang closed forms of the 2D Ising model.
bruteforce    exact contraction of small finite networks.

Parity status of every function is recorded in its docstring; a function
without an external pin says "parity unpinned".
"""
