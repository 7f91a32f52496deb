"""MI355X (gfx950) staggered Dslash and even-odd CG: Python binding of liblgt.so.

Argument marshalling only: every step runs in the HIP kernels of liblgt.so
(see include/lgt.h for the operation, layouts and error behaviour). Device
memory and the stream come from PyTorch; if the shared library is missing,
importing this package raises at once -- there is no fallback path.
"""
from __future__ import annotations

from .lgt import (  # noqa: F401
    LGT_BF16, LGT_F32, LGT_F64, LGT_R12, LGT_R18, LGT_EVEN, LGT_ODD,
    LGT_CG_FP64, LGT_CG_RELIABLE, LGT_CG_REFINE, STATUS,
    LGT_MRHS_LANE, LGT_MRHS_VALU4, LGT_MRHS_MFMA, LgtError,
    Lattice, PackedLinks, CgResult, PseudofermionAction, ImprovedPseudofermionAction, cg_solve_batch, routine, ROUTINES, PLANES,
    asqtad_coeffs,
    lib, lib_path, exported_symbols, links_bytes, vec_bytes, geom_check,
    DSLASH_FLOP_PER_SITE, IMPROVED_FLOP_PER_SITE, link_bytes_per_dir, vec_bytes_per_site,
)

lib()  # load liblgt.so now: a missing library fails the import, not a later call
