"""MI355X-native MONC advection: PW momentum + ULTIMATE/TVD scalars in HIP.

The C ABI lives in include/monc_adv.h and libmoncadv.so (built in-tree by
paper_2009_12850_amd.build); _lib is the thin ctypes binding with the same
names; inputs holds the seeded synthetic input generators.
"""
from . import _lib  # noqa: F401
from ._lib import (MONC_BF16, MONC_F32, MONC_F64, MONC_NBUDGET, MoncError,  # noqa: F401
                   budgets_dict, monc_advect, monc_advect_pw, monc_advect_tvd,
                   monc_budgets_check, monc_cast_working, monc_halo_fill, monc_step,
                   monc_step_mixed, monc_step_workspace_bytes)
