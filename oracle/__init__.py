"""Plain FP64 CPU oracle for the multiple-scattering operator in a two-layer
elastic medium (Zhang, He, Lai, "A fast solver for many-particle elastic
scattering in layered media").

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call this package.  It shares
no code with the HIP library and never imports it.

What it computes (paper frame: particles in y < 0, interface y = 0):

* ``media``        wavenumbers (Section 2, Helmholtz split; density kept).
* ``smatrix``      closed-form disk scattering matrices, rigid and
                   traction-free (Section 4.1), and basis rotation (Section 4.3).
* ``graf``         dense O(N^2) free-space translations (Section 4.2, Graf).
* ``interface``    the per-node 2x2 P-SV reflection of the welded interface
                   (Section 3.2, the 4x4 system solved per Fourier mode).
* ``sommerfeld``   the layered reflected part: multipole-to-Sommerfeld
                   (Lemma, Section 5.4), reflection, Sommerfeld-to-local
                   (Jacobi-Anger, Section 5.3), integrated by adaptive
                   Gauss-Kronrod quadrature on the real axis.
* ``incident``     plane-wave right-hand side (Section 7.3).
* ``operator``     y = x - S (T_free + T_refl) x, the Schur-complement operator
                   of Section 5.2, and its conjugate transpose.
* ``gmres``        textbook GMRES (Saad-Schultz) with CGS2 Arnoldi.
* ``field``        scattered displacement at receivers (Section 5, coupled
                   representation).

* ``shapes``       scattering matrices of ellipses, stars and the paper's pear
                   and starfish by fundamental solutions (Section 4.3).

Each part is pinned by the tests in ``tests/test_oracle_*.py`` (closed forms,
invariants, brute force), except one: parity unpinned for the non-circular
S-matrices of ``shapes`` (no closed form; pinned only by the disk limit,
unitarity, the boundary condition between collocation points, rotation and
convergence in the point count).
"""
from . import media, smatrix, graf, interface, sommerfeld, incident, operator, gmres, field  # noqa: F401
from .media import Media, wavenumbers  # noqa: F401
