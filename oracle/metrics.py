"""Error measures.  TEST INFRASTRUCTURE ONLY (see the package docstring)."""
from __future__ import annotations

import numpy as np


def l1_rel_error(num, ref) -> float:
    """Relative L1 error of Sec. VI: sum |x_num - x_ref| / sum |x_ref|."""
    num = np.asarray(num, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.abs(ref).sum()
    return float(np.abs(num - ref).sum() / den) if den > 0 else float(np.abs(num - ref).sum())
