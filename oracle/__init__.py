"""CPU oracle for the thin-disk B-spline self-gravity method (arXiv 1904.07400).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute
anything under ``oracle/``.  The product path (``paper_1904_07400_amd``) never
does, and the two share no code: no kernels, headers, helpers, tables or
constant generators.  Inputs come from the separate ``workloads`` module,
which holds none of the method's arithmetic.

Everything here is plain FP64 on the CPU and uses no FFT:

* ``sample_lattice``     - where sigma is sampled for order k (Sec. 2.2, Sec. 2.3)
* ``bspline_coeffs``     - sigma -> C by the two tridiagonal systems of
                           Eqs. (z_system) and (C_system), Thomas algorithm;
                           k = 4, 5 by the banded systems of the same
                           construction (LAPACK banded LU)
* ``weights``            - w^x, w^y of Eq. (eqnwB) by quadrature of their
                           defining integral (C code, ``csrc/sg_oracle.c``)
* ``forces``             - F = C * w by direct summation, Eq. (eqnF)
* ``forces_adjoint``     - the transpose of sigma -> (Fx, Fy)
* ``disk_force_radial``  - analytic F_R of the D3 / D4 disks (Sec. 3)
* ``error_norms``        - L1 / L2 / Linf of Eqs. (oneNormErr)-(inftyNormErr)
* ``antiderivative``     - the closed forms of Appendix A and Eq. (intF) (mpmath)

Where the paper is silent or ambiguous the oracle takes these readings: the
k = 2 and k = 4 splines are centred on the vertices x0 + i dx and sampled
there; the k = 3 and k = 5 labels are shifted so that C_i is centred on cell i; the weight
integral over the piece holding the singular point is a principal value;
the error norms are weighted by the cell area; G = 1 and the force is
attractive.
"""
from .core import (  # noqa: F401
    sample_lattice, cell_centres, thomas, banded_solve, STENCIL, bspline_coeffs, bspline_apply, bspline_value,
    weights, weights_at, forces, forces_from_coeffs, forces_sparse, forces_adjoint,
    coeffs_transpose_solve, disk_force_radial, error_norms, accuracy_order,
    antiderivative, antiderivative_intF, build,
)
