"""CPU oracle for the elevation-map fusion path (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does.  The two
share no code, headers, helpers or constants.
"""
from .elevation import *  # noqa: F401,F403
from .elevation import __all__ as _all_elevation
from .filters import *  # noqa: F401,F403
from .filters import __all__ as _all_filters

__all__ = list(_all_elevation) + list(_all_filters)
