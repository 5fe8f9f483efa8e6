"""MI355X-native differentiable propagation of superconducting-qubit systems.

The compute path is the HIP library ``libscprop.so`` (built in-tree by
``build_lib.build``); this package is its Python binding.  Importing the
package loads the library and fails loudly when it has not been built.
"""
from ._lib import ScpError, lib  # noqa: F401

lib()  # fail loudly if the HIP library is missing

from .api import (ChannelTarget, StateTarget, System, Target, basis_columns,  # noqa: E402,F401
                  fidelity, fidelity_channel, fidelity_local, fidelity_states, fidelity_zcomp,
                  matrix_units, padded_indices, probe_contraction)
from . import autograd  # noqa: E402,F401
