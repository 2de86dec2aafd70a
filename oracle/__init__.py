"""CPU FP64 oracle for the T-matrix multiple-scattering hot path.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check in __graft_entry__ and
the cpu_baseline leg of bench.py may import this package.  It shares no code
with the HIP path (paper_2107_09879_amd) and never imports it; the two meet
only in the seeded input generators of the `workloads` package.

It is a plain, slow, double-precision implementation written from the paper's
App. I (T-matrix method), App. II (plane-wave expansion) and App. IV (adjoint),
with the readings listed in each module docstring.
"""
from .mie import mie_ab, mie_tmatrix_diag, mie_tmatrix_diag_many  # noqa: F401
from .solver import (LatticeCoupling, coupling_dense, detector_vectors,  # noqa: F401
                     extinction, far_field, gmres, near_field,
                     objective_and_gradient_dense, rows_A, scattering,
                     solve_dense, system_dense, tmatrix_dense)
from .position import (detector_vector_gradient, objective_and_position_gradient_dense,  # noqa: F401
                       objective_dense, translation_gradient)
from .translation import Translation, ab5  # noqa: F401
from .vswf import (index_list, n_coeffs, plane_wave_angular,  # noqa: F401
                   plane_wave_coeffs, vswf, vswf_farfield)
