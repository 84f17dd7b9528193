"""Plain, slow, FP64 CPU oracle for symmetry-reduced light-cone QAOA MaxCut energies.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product path (the C-ABI library and its Python binding) never imports, links or
calls it, and shares no code, header, table or helper with it.

The oracle follows the paper (Shaydulin & Wild, "Exploiting Symmetry Reduces the Cost
of Training QAOA", arXiv:2101.10296) step by step:

* ``problem``     - MaxCut input: G=(V,E), optional weights J (Sec. 2.4; Sec. 4, Eq. 6)
* ``orbits``      - equivalence classes of Hamiltonian terms under a supplied group of
                    graph automorphisms, by explicit closure (Sec. 2.6; Sec. 3, Thm. 1
                    and the reduced-energy display)
* ``cones``       - reverse causal cone of a term: the radius-p ball around its two
                    endpoints (Sec. 2.3)
* ``statevector`` - the QAOA state on a cone, its <Z_u Z_v> and a forward-mode gradient
                    (Sec. 2.2 ansatz; Sec. 2.3 per-term decomposition)
* ``energy``      - orbit-weighted energy and the plain unreduced sum (Sec. 3), full-graph
                    brute force, central finite differences
* ``closed_form`` - the p=1 closed form of a MaxCut edge term (a published result the
                    paper relies on implicitly; used as an independent pin)
* ``automorphisms`` - brute-force automorphism groups of tiny graphs (Sec. 2.6-2.7)
* ``train``       - Adam ascent of the oracle energy over a batch of starting angles
* ``rqaoa``       - recursive QAOA (pair elimination) with oracle correlations

Every function works in float64 / complex128.  Every pin that fixes this code against
the paper or the mathematics lives in ``tests/test_oracle_*.py``.
"""
from .problem import canonical_edges  # noqa: F401
from .orbits import edge_orbits  # noqa: F401
from .cones import light_cone  # noqa: F401
from .statevector import cut_values, qaoa_state, zz_expectation, zz_and_grad  # noqa: F401
from .energy import plan, energy, energy_grad, energy_fd, bruteforce_full  # noqa: F401
from .closed_form import zz_p1  # noqa: F401
from .automorphisms import automorphism_group, group_closure  # noqa: F401
from .train import adam_ascent  # noqa: F401
from . import rqaoa  # noqa: F401
