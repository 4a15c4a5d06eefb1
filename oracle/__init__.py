"""Oracle for InfraredGP's feed-forward propagation (FFP).

TEST INFRASTRUCTURE ONLY.  A plain, slow, FP64 CPU statement of what the GPU
path computes, written from the paper (arXiv 2508.19737): the degree-corrected
Laplacian (Sec. I and Eq. (1)), the low-pass filter (Eq. (2)), its spatial form
(Eq. (3)), the layer (Eq. (4)) and the static procedure (Algorithm 1, steps up
to the final sigmoid).  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import anything from this package; the
product library never does, and this package imports nothing from it.

Modules
  ffp     sparse FP64 reference of the whole FFP (CSR build, D_tau, scales,
          counter-based Gaussian input, hops, ZNorm, sigmoid)
  dense   dense brute force for tiny graphs: eigendecomposition of L_tau,
          the spectral filter, Gershgorin discs
  cref    ctypes loader for the plain-C FP64 FFP (cpu_ref.c), same math,
          used where the NumPy version is too slow (millions of nodes)

Parity status of each function is stated in its docstring; every function is
pinned by a CPU test against facts the paper or mathematics fixes, except the
Gaussian input's correspondence to the paper's own (unknown) random draw,
which is "parity unpinned" by nature: the paper does not say which generator
it used.
"""
