"""Plain FP64 CPU oracle for the constant-potential electrode-charge step.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything here; the
product path (the C-ABI library and its Python binding) never does. The
oracle shares no code with the GPU path: the only module both import is the
seeded workload generator, which holds none of the method's arithmetic.

Every function follows a passage of the paper (Li, Wang, Liu, Jiang, "A
simple and efficient lattice summation method for metallic electrodes in
constant potential molecular dynamics simulation", arXiv 2111.06704) and
cites it by section / equation. Notation used here: ``a`` is the Gaussian
inverse width of an electrode charge (the paper's alpha_i), ``beta`` is the
Ewald splitting parameter (the paper's eta). Units: Gaussian electrostatic
units with lengths in Angstrom, so matrix entries are in 1/A and potentials
are in e/A; volts convert with k_e = e^2/(4 pi eps0).

Modules:
  ewald    - k-vector set, the Gaussian Ewald matrix E (Eq. 22-23), the
             electrolyte potential b_sol (Eq. 25) and a matrix-free
             potential evaluation (Eq. 21); for systems too large for the
             direct phase sums (N = 131072 with 200000 ions) the same
             structure factors and reciprocal sums through per-axis factors
             of exp(i K.r) and complex matrix products, pinned to the direct
             routines.
  cpm      - the constrained solve: Cholesky, neutralising vector (S8-S9),
             two-step neutralisation (Eq. 35), bordered Lagrange system
             (Eq. 29) and the S matrix (Eq. 33); the matrix-inversion
             construction E = U Q^-1 (S10-S13).
  features - per-atom warm-start features (12 nearest neighbours).
  mlp      - FP64 multilayer perceptron, its gradient and the Adam step.

Parity status: every function is pinned by a test under tests/ except the
choice of network minimiser reached by training (parity unpinned: which
local minimum training reaches is not fixed by anything; the network's
forward pass, gradient and optimiser step are pinned).
"""
