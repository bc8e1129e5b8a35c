"""MI355X (gfx950) implementation of the Monte Carlo Kolmogorov-Smirnov method
for fitting the discrete power law (Rappos & Robert, 2013): HIP kernels behind
the C ABI of include/zpl.h, with a thin ctypes binding (``zpl``)."""
from .zpl import (CellSpec, Context, ZplError, FLAG_ALL_ONES, FLAG_BISECT,  # noqa: F401
                  FLAG_NOCONV, FLAG_TAIL_CAPPED, TABLE_H, exported_symbols, lib,
                  cell_array, load_tuning, plan_forms, save_tuning)
