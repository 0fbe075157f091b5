"""ctypes loader of the plain C CIC deposit (oracle/cic.c).

TEST INFRASTRUCTURE ONLY, like the rest of this package.  ``deposit_c``
computes exactly what ``cwthf.deposit`` computes (Sec. 2 step 2, Eq. (1)), for
boxes whose particle count NumPy's add.at cannot handle in reasonable time.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .cwthf import DepositOverflow

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cic.c")
LIB = os.path.join(HERE, "libcic.so")

_lib = None


def build() -> str:
    """Compile cic.c with gcc: no FMA contraction, no fast-math, so every
    multiply is the single correctly rounded operation the definition asks for."""
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
                    "-o", tmp, SRC, "-lm"], check=True, capture_output=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        for name in ("oracle_cic_deposit_f32", "oracle_cic_deposit_f64"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                          ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
        _lib = lib
    return _lib


def deposit_c(pos: np.ndarray, box_len: float, n: int, frac_bits: int = 15, threads: int = 1) -> np.ndarray:
    """The CIC density of ``cwthf.deposit``, int64 [n][n][n], from the C loop.
    With threads > 1 the z planes are split into that many contiguous ranges,
    each filled by its own call (every call reads all particles)."""
    pos = np.ascontiguousarray(pos)
    if pos.dtype not in (np.float32, np.float64):
        raise TypeError("positions must be float32 or float64")
    if pos.ndim != 2 or pos.shape[1] != 3:
        raise ValueError("positions must have shape [np, 3]")
    if not 8 <= frac_bits <= 20:
        raise ValueError("frac_bits must be in [8, 20]")
    rho = np.zeros((n, n, n), dtype=np.int64)
    f = _load().oracle_cic_deposit_f32 if pos.dtype == np.float32 else _load().oracle_cic_deposit_f64
    k = max(1, min(int(threads), n))
    bounds = [(n * i) // k for i in range(k + 1)]

    def run(i):
        return f(pos.ctypes.data, pos.shape[0], float(box_len), int(n), int(frac_bits), bounds[i], bounds[i + 1],
                 rho.ctypes.data)

    if k == 1:
        codes = [run(0)]
    else:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=k) as ex:
            codes = list(ex.map(run, range(k)))
    if 1 in codes:
        raise ValueError("non-finite or out-of-range particle position")
    if 2 in codes:
        raise DepositOverflow("a CIC cell exceeds 2^63 - 1")
    return rho
