"""Plain FP64 CPU oracle of the multi-rhs HISQ Dslash and the even-odd CG solve.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The GPU path neither imports it nor shares any code with it;
the only thing both sides share is the seeded input generator in ``synth``.

Every function here is the plain definition written out with numpy, in float64/complex128, with
no blocking, fusion or reordering beyond what the definition states.  Each cites the passage of
Kaczmarek et al., "HISQ inverter on Intel Xeon Phi and NVIDIA GPUs" (PoS LATTICE2014), that it
follows.  The pins that tie these functions to the paper and to mathematics independent of this
code are in tests/test_oracle_pins.py, test_oracle_fcg.py, test_oracle_nn.py and
test_oracle_trace.py; tests/test_oracle_mutations.py checks that planted slips in a copy of this
package fail them.

Parity status: every function here is pinned (closed forms, invariants, dense LU, finite
differences), see the pin tests.
"""
from .dslash import (  # noqa: F401
    dslash_full, dslash_half, dslash_sites, embed, extract, m_ee, parity_lex, site_coords,
)
from .cg import cg, fcg, true_residual  # noqa: F401
from . import nn  # noqa: F401
from . import trace  # noqa: F401
