"""FP64 CPU oracle for one semi-implicit pseudo-spectral step of dilute-polymer
plane-channel flow (Oldroyd-B / sPTT conformation tensor, no positivity
enforcement).

TEST INFRASTRUCTURE ONLY.  This package exists to check the HIP library
against an independent, plain, slow implementation of the same discrete
problem.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The product path
(``paper_2606_09468_amd``) never imports, links or executes anything here,
and nothing here imports the product package.

What is computed (paper, Section 2):
  * eq. (1): conformation tensor c, transported by u, stretched by the velocity
    gradient, relaxed towards I over the time Wi, with polymer diffusion kappa
    and the sPTT factor [1 + eps Tr(c - I)];
  * eq. (2): momentum with solvent viscosity beta/Re, polymer stress
    divergence (1 - beta)/(Re Wi) div c and a streamwise drive;
  * eq. (3): incompressibility;
  * walls y = +-1 with no slip; conformation wall values from eq. (1) with
    kappa = 0 (Section 2, boundary-condition paragraph);
  * Fourier in x and z, Chebyshev in y, fully dealiased (Section 2, numerics
    paragraph).
The discrete choices the paper leaves open (collocation grid, 3/2 padding in
y, velocity-vorticity form with influence matrix, CNAB2 in place of the
paper's 4th-order BDF, constant flux, initial perturbation) are listed with
their readings in the repository's design notes; each function here names the
part of the paper it follows.

Modules:
  cheb      Chebyshev Gauss-Lobatto grid and operators (extended precision,
            rounded once to float64)
  fourier   padded Fourier transforms in x and z (numpy.fft, float64)
  initial   laminar Poiseuille base state and the seeded perturbation
  channel   the Oracle class: state, explicit terms, CNAB2 step, diagnostics
  stats     midplane statistics: histogram of the samples, P(Tr c < 3), chi
  resample  a state carried to another resolution (spectral pad/truncate)
"""

from .channel import Oracle, Grid, Params, state_layout  # noqa: F401
from . import stats  # noqa: F401
from . import resample  # noqa: F401
