"""CPU complex128 oracle for the sound-soft multiple-scattering hot path of
mu-diff (Thierry, Antoine, Chniti, Alzubaidi, arXiv:1409.8186).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The HIP library
and its Python binding never import, call or link anything here, and this
package imports nothing from them: the two share no code.

What it computes, each module citing the paper passage it writes out:

  geometry   disk/pair geometry b_pq, alpha_pq, mode offsets      (sec. 4.1, sec. 5)
  bessel     J_m, H_m^(1) and derivatives at integer orders       (sec. 4.2; SciPy/AMOS)
  operator   dense truncated EFIE matrix L, its diagonal D,       (sec. 4.2 block formulas,
             the single-scattering preconditioned A = D^-1 L       sec. 5 system and
                                                                   preconditioner)
  rhs        plane-wave Fourier coefficients U                    (Prop. 4)
  farfield   far-field row vectors g(theta) and a = g^T rho       (sec. 4.4)
  solve      dense LU solve of L rho = -U, restarted GMRES(m)     (sec. 5)
  gradient   far-field misfit, its adjoint gradient w.r.t.
             centers, radii and k, and central differences        (derived from sec. 4-5)
  operators  the operators M, N, D and identity, combinations,    (sec. 3 formulations,
             normal-derivative plane-wave coefficients, the        sec. 4.2 block formulas,
             double-layer far field; EFIE, MFIE, CFIE, BWIE,        Prop. 4, sec. 4.4)
             sound-hard single- and double-layer equations
  penetrable transmission problem of penetrable disks: the 2x2       (sec. 7, Example II)
             block system, far field, interior fields
  pointsource trace coefficients of a point source's incident wave  (Prop. 5)
             and the incident field (i/4) H_0(k |x - s|)
  nearfield  single- and double-layer potentials at points        (sec. 4.4, Graf's theorem)
             and the total field
  dort       far-field mirror matrix F, time-reversal matrix      (sec. 7, Example III)
             T = conj(F)^T F, its eigen-decomposition, Herglotz waves

Everything is float64 / complex128, written as the plain definition: dense
matrices, library LU and Bessel routines, no blocking, fusion or reordering.
Every function is pinned by a ``-m "not gpu"`` test against something other
than itself (closed forms, quadrature of the defining integrals, exact
identities of the truncated system, brute force).  The one output with no
such pin is the GMRES iteration count (parity unpinned; the converged
solution is pinned against LU).
"""
from . import geometry, bessel, operator, rhs, farfield, solve, gradient, dort, operators, nearfield, penetrable, pointsource  # noqa: F401
