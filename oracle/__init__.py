"""Plain FP64 CPU oracle for the staggered spectral semi-implicit DG pressure path
(Fambri & Dumbser, arXiv:1602.05806, Section "Spectral semi-implicit DG schemes on
staggered Cartesian grids").

THIS PACKAGE IS TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it. The product path (the HIP library and its
Python binding) never imports, links or calls anything here, and nothing here imports the
product path. The two share no code: the 1D reference-element tables, the assembled operators
and the solvers below are computed independently of the C++/HIP library.

Everything is written for a reader who has the paper open: each function names the equation
or section it follows. Blocking, fusion or reordering beyond the paper's definitions is
deliberately absent; speed is not a goal.

Modules
-------
basis      1D Gauss-Legendre nodal basis and the 1D matrices of eq. (matrices), the L2
           projection matrices of eq. (l2forward), and the pressure blocks of eq. (pSyst).
layout     conversion between the element-blocked DoF layout of the library boundary and the
           tensor layout used for Kronecker assembly.
operators  assembled sparse operators: weak gradient D (eq. weakgradientop), H = D^T M^-1 D
           (eq. PerPrSyst), the pressure and viscous operators, the divergence RHS map and the
           null space of D.
solvers    Hestenes-Stiefel CG, dense Cholesky of A + Z Z^T, and a fast-diagonalisation direct
           solver (exact minimum-norm solution on periodic grids).
step       the fractional step of eqs. (LOdiffusionU)-(LOvelocityW): L2 projections,
           Rusanov DG convection with third-order TVD Runge-Kutta, viscous and pressure solves,
           velocity update.
adjoint    transposed operators of the step (dot-product pins) and the discrete adjoint.
"""
