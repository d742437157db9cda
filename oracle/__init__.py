"""CPU FP64 oracle for the hierarchical standard-siren log-likelihood.

TEST INFRASTRUCTURE.  This package is the plain, slow, obviously correct
reference that the HIP library is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with ``paper_2504_02034_amd`` (the library, its
binding and its preprocessing) and imports nothing from it; both sides are fed
by the same seeded raw inputs only.

Every function follows a passage of Tagliazucchi, Moresco, Borghi & Fiebig
(2025), "Accelerating the standard siren method" (arXiv:2504.02034), cited by
section and equation label.  Where the paper is silent the reading taken is
stated in the docstring; the list of readings is kept with the design notes.

Modules
-------
cosmology   flat-LCDM distance (eq. dL-em), Xi0-n ratio (eq. dL-mg), its
            z-derivative (the Jacobian of eq. jacobian), inversion d -> z
population  power-law + Gaussian-peak mass model and Madau-Dickinson rate
            (Sect. 3.1)
likelihood  bandwidth, many-1D KDE (eq. gw-kernel-many1d), per-event
            integrals (eq. like-integrals), injection estimator of xi
            (Sect. 2.2), ln L (eq. hyperlike)
prep        the lambda-independent pre-computation (Sect. 2.3 steps a-c):
            region, 2-D sky factors, catalogue density on the grid (eq. p-cat)
gradient    d lnL / d lambda by the chain rule, and finite differences

Parity status per function is listed in each module header; functions with
no independent pin say "parity unpinned".
"""
from . import cosmology, population, likelihood, prep, gradient  # noqa: F401
