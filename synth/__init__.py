"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package holds input generators only: argon-shaped cross-section tables,
workload parameter sets and seeded marker states.  It performs none of the
simulation method's arithmetic (no push, no collision sampling, no deposit,
no field solve), so both sides of every parity test can take their inputs
from here without sharing any of the computation they are checked on.
"""

from .xsec import CrossSections, argon_like, argon_five, fixed_event  # noqa: F401
from .constants import (QE, KB, ME, AMU, M_AR, EPS0, TORR,  # noqa: F401
                        gas_density)
from . import configs, markers  # noqa: F401
