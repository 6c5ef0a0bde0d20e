"""Plain FP64 CPU oracle for the PNOF5 / PNOF7 / PNOF7s orbital-optimisation step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or load
this package: it is used by ``tests/``, by the smoke check and by the
``cpu_baseline`` leg of the benchmark, and it shares no code with the device
library (``paper_2004_06142_amd``).  Its inputs come only from ``synth``.

Every function follows the passage of Piris & Mitxelena, "DoNOF: an open-source
implementation of natural-orbital-functional-based methods for quantum
chemistry" (arXiv:2004.06142) that its docstring cites, in float64, with no
blocking or reordering beyond what the definition states.  Two routes exist:

* ``oracle.pnof``    the definitional route: per-orbital AO matrices J^q, K^q, F^q
                     materialised as written in Section 3.5 (Eqs. JKpq, Gpmn) and
                     Section 3.2 (Eqs. lowdin, Vee-s, Vee-d, lag);
* ``oracle.stream``  the same quantities as a loop over density-fitting rows P,
                     for sizes where J^q, K^q cannot be materialised.

Parity status: every function is pinned by tests in ``tests/test_oracle_*.py``
(brute force, closed forms, special cases, finite differences).  The PNOF7
Phi-term has no generating wavefunction; it is pinned by the explicit
two-particle reduced density matrix route (Eqs. intra, interaa, interab), the
half-filling identity with PNOF7s, the Hartree-Fock limit and finite differences.
"""
from . import pnof, stream  # noqa: F401
