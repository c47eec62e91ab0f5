"""FP64 CPU oracle for the plane-wave H*psi + Chebyshev-filtered subspace path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The library under
``paper_2507_08578_amd`` never imports it and shares no code with it; the
two meet only through the seeded inputs of ``synth``.

Everything here is plain numpy/scipy in float64/complex128, written to be
checked against the paper by eye: no blocking, fusion or reordering beyond
what each definition states.
"""
from .pw_oracle import (  # noqa: F401
    kinetic, scatter_to_box, gather_from_box, fft_backward, fft_forward,
    dft_backward_direct, dft_forward_direct, apply_local, apply_nonlocal, apply_h,
    dense_h, upper_bound, cheb_filter, cheb_filter_closed_form, orthonormalize,
    rayleigh_ritz, chfsi, OracleHam, cell_volume, density, density_at,
)
from . import eigensolvers  # noqa: F401,E402
from .eigensolvers import (  # noqa: F401,E402
    teter_factor, band_kinetic, precondition, block_bounds, lobpcg, line_step, rmm_diis,
    LobpcgResult, RmmDiisResult,
)
