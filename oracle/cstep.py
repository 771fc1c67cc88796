"""Sequential implicit Euler with Jacobi-PCG, in plain C with OpenMP (oracle side).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.  ``seqstep.c`` takes the
CSR matrix that :func:`oracle.fv.assemble_linear` builds and steps
``(I/tau + K) y^{n+1} = y^n / tau + b`` (implicit Euler, the one-stage tableau of
Sec. 2, eq. stiffly-accurate-DIRK) one solve per step, stopping each solve at
``||rhs - J y|| <= rtol ||rhs||``.  It exists because the scipy form
(:func:`oracle.stepping.dirk_linear`) runs one core only: at 2 million cells the C
form checks full-size runs in seconds, and times the oracle on every host core.

``build()`` compiles ``seqstep.c`` with gcc into ``oracle/libseqstep.so``;
``ie_steps`` builds it on first use when it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "seqstep.c")
LIB = os.path.join(HERE, "libseqstep.so")
_lib = None


def build() -> str:
    """Compile the C oracle (gcc, OpenMP, no machine-specific flags) and return the library path."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99", SRC, "-o", tmp, "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"oracle C build failed: {' '.join(cmd)}\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        lib.orc_ie_steps.restype = ctypes.c_int
        lib.orc_ie_steps.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_double, P, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_int, P, P, P]
        _lib = lib
    return _lib


def ie_steps(K, b, y0, tau, n_steps, rtol=1e-12, maxit=200000, threads=0):
    """Implicit Euler for ``y' + K y = b`` from ``y0``: ``n_steps`` steps of size ``tau``.

    ``K`` is a scipy CSR matrix, ``b`` a vector or ``None``.  ``threads`` = 0 uses the
    OpenMP default (every core).  Returns ``(ys, iters, threads_used)``: ``ys[n]`` is
    ``y^n`` with ``ys[0] = y0`` (a list of arrays), ``iters`` the CG iterations per step.
    """
    lib = _load()
    K = K.tocsr()
    K.sort_indices()
    N = K.shape[0]
    rp = np.ascontiguousarray(K.indptr, dtype=np.int32)
    ci = np.ascontiguousarray(K.indices, dtype=np.int32)
    va = np.ascontiguousarray(K.data, dtype=np.float64)
    bb = None if b is None else np.ascontiguousarray(b, dtype=np.float64)
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    ys = np.empty((n_steps, N), dtype=np.float64)
    its = np.zeros(n_steps, dtype=np.int32)
    used = ctypes.c_int(0)
    st = lib.orc_ie_steps(N, rp.ctypes.data, ci.ctypes.data, va.ctypes.data,
                          None if bb is None else bb.ctypes.data, float(tau), y0.ctypes.data, int(n_steps),
                          float(rtol), int(maxit), int(threads), ys.ctypes.data, its.ctypes.data,
                          ctypes.byref(used))
    if st != 0:
        raise RuntimeError(f"oracle C stepping failed (status {st})")
    return [y0.copy()] + [ys[i] for i in range(n_steps)], its.tolist(), used.value
