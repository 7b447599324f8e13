"""CPU FP64 oracle for the FFT-preconditioned FE homogenization solver.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this package.  It shares no code,
tables or constants with the HIP library and imports nothing from it.

The oracle computes the definitions of the paper directly, with plain,
slow, independent algorithms:

  * Sec. 3 (eqs. Du_mat, grad_componets, W_mat, lin_system): the stiffness
    K = D^T W C D is *assembled* as a sparse CSR matrix from element
    matrices built from the shape-function gradients at the quadrature
    points (elements.py, assembly.py);
  * Sec. 4.1-4.2 (eqs. Kref, M, M_inverse) and Sec. 5.2-5.3 (Alg. 2): the
    reference-material preconditioner is the Moore-Penrose pseudo-inverse of
    Kref applied through a *naive* (matrix, not fast) unnormalised DFT of the
    impulse-response column of the assembled Kref (naive_dft.py, precond.py);
  * Alg. 1 with a linear material (one Newton step from u0 = 0) and the
    relative Kref^-1-norm stopping rule of Sec. 6 (pcg.py);
  * the homogenized tensor as the energy (bilinear) form over quadrature
    points, and the stress average as a diagnostic (homog.py);
  * PCG from an initial guess u0 (the starting point of Alg. 1) with the
    warm-start screen (pcg.py), and the learned warm start's network, loss
    and Adam step in FP64, optionally rounding stored tensors to BF16 as
    the GPU stores them (convnet.py).

Every function cites the passage it follows.  See pins in
tests/test_oracle_pins.py for what fixes each part independently.
"""
from .elements import element  # noqa: F401
from .assembly import Problem, assemble_stiffness, rhs, element_matrix  # noqa: F401
from .naive_dft import dft, idft  # noqa: F401
from .precond import reference_symbol, pseudo_inverse_blocks, Preconditioner  # noqa: F401
from .pcg import pcg  # noqa: F401
from .homog import homogenize, homogenized_energy, mean_material, stress_average  # noqa: F401
