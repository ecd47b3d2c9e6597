"""CPU oracle for the hafnian / loop hafnian -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it, and it
shares no code with the GPU library (the seeded input generators live in
``gen/``, which holds none of the method's arithmetic).

Routes (see ``haf_oracle.c`` for the arithmetic):

* ``brute``          -- the definitions (Sec. 2, Eq. hafA; the loop-hafnian sum
                        over single-pair matchings), long double, n <= 24;
* ``brute_int``      -- the same, exact 128-bit integers, for integer matrices;
* ``formula``        -- the inclusion-exclusion sum of Sec. 3.2 with f(Z) from
                        Sec. 3.3 (Eq. poly, Eq. haffinal and the loop formula),
                        power traces from explicit matrix powers; precision
                        ``"d"``, ``"ld"``, ``"dd"`` or ``"q"``;
* ``modp``/``exact_int`` -- the same sum over F_p and a CRT reconstruction
                        (each f(Z) counts tangles, Sec. 3.2, so it is an integer);
* ``ryser``          -- permanents, for the bipartite identity (Sec. 1.1).

Readings of the paper that this oracle fixes:
the loop term is d^T B^(k-1) (X d) with B built from the zero-diagonal matrix
(the printed v (XB)^(k-1) v^T fails already at n = 2); pairs are (2i, 2i+1),
i = 0..n/2-1; n = 0 gives 1; odd n gives haf = 0 and lhaf through padding
with an isolated loop of weight 1.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_haf_oracle.so")
_SRC = [os.path.join(_HERE, "haf_oracle.c"), os.path.join(_HERE, "formula_body.inc")]

PREC = {"d": 0, "ld": 1, "dd": 2, "q": 3}
EPS = {"d": 2.0 ** -53, "ld": 2.0 ** -64, "dd": 2.0 ** -104, "q": 2.0 ** -113}


def build(force: bool = True) -> str:
    """Compile the oracle library with gcc (it is plain C + OpenMP)."""
    if not force and os.path.exists(_SO) and all(
        os.path.getmtime(_SO) >= os.path.getmtime(s) for s in _SRC
    ):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC[0],
           "-lquadmath", "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.orc_formula_range.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                          ctypes.c_uint64, ctypes.c_int, dp, dp]
        lib.orc_formula_masks.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, u32p, ctypes.c_int64,
                                          ctypes.c_int, dp]
        lib.orc_term.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint32, dp]
        lib.orc_ryser.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        lib.orc_brute.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp]
        lib.orc_brute_int.argtypes = [i64p, ctypes.c_int, ctypes.c_int, u64p]
        lib.orc_modp.argtypes = [i64p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, u64p]
        lib.orc_modp_term.argtypes = [i64p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, u64p]
        for f in (lib.orc_formula_range, lib.orc_formula_masks, lib.orc_term, lib.orc_ryser, lib.orc_brute,
                  lib.orc_brute_int, lib.orc_modp, lib.orc_modp_term):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _cplx(A) -> np.ndarray:
    A = np.ascontiguousarray(np.asarray(A, dtype=np.complex128))
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("expected a square matrix")
    return A


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class HighPrec:
    """A complex value carried as (hi, lo) double pairs per component."""

    __slots__ = ("re_hi", "re_lo", "im_hi", "im_lo")

    def __init__(self, out):
        self.re_hi, self.re_lo, self.im_hi, self.im_lo = (float(x) for x in out)

    @property
    def value(self) -> complex:
        return complex(self.re_hi + self.re_lo, self.im_hi + self.im_lo)

    def exact_parts(self):
        return (Fraction(self.re_hi) + Fraction(self.re_lo), Fraction(self.im_hi) + Fraction(self.im_lo))

    def relerr(self, z: complex) -> float:
        """|z - self| / |self|, evaluated with the lo parts kept."""
        re, im = self.exact_parts()
        dr = Fraction(z.real) - re
        di = Fraction(z.imag) - im
        num = float(dr) ** 2 + float(di) ** 2
        den = float(re) ** 2 + float(im) ** 2
        return (num / den) ** 0.5 if den else float(num ** 0.5)

    def relerr_hp(self, other: "HighPrec") -> float:
        """|other - self| / |self| with both lo parts kept."""
        re, im = self.exact_parts()
        ore, oim = other.exact_parts()
        num = float(ore - re) ** 2 + float(oim - im) ** 2
        den = float(re) ** 2 + float(im) ** 2
        return (num / den) ** 0.5 if den else float(num ** 0.5)

    def __repr__(self):
        return "HighPrec(%r)" % (self.value,)


def _pad_odd(A: np.ndarray, loops: bool):
    """Odd n: haf is 0 (no perfect matching); lhaf equals lhaf(A (+) [1])."""
    n = A.shape[0]
    if n % 2 == 0:
        return A, False
    if not loops:
        return None, True
    B = np.zeros((n + 1, n + 1), dtype=np.complex128)
    B[:n, :n] = A
    B[n, n] = 1.0
    return B, False


def brute(A, loops: bool = False) -> HighPrec:
    """haf or lhaf from the definition (long double), n <= 24."""
    A = _cplx(A)
    out = np.zeros(4)
    if _load().orc_brute(_dptr(A), A.shape[0], int(loops), _dptr(out)) != 0:
        raise ValueError("brute force: n out of range")
    return HighPrec(out)


def brute_int(A, loops: bool = False) -> int:
    """Exact haf/lhaf of an integer matrix from the definition, n <= 24."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.int64))
    out = np.zeros(2, dtype=np.uint64)
    rc = _load().orc_brute_int(A.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), A.shape[0], int(loops),
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if rc != 0:
        raise ValueError("brute_int: n out of range")
    v = int(out[0]) | (int(out[1]) << 64)
    if v >= 1 << 127:
        v -= 1 << 128
    return v


def formula(A, loops: bool = False, prec: str = "ld", threads: int | None = None, want_kappa: bool = False):
    """The subset-sum formula (Sec. 3) with explicit-power traces.

    Returns a HighPrec, or (HighPrec, kappa) with kappa = sum_Z |f(Z)| / |result|.
    """
    A = _cplx(A)
    Ap, zero = _pad_odd(A, loops)
    if zero:
        r = HighPrec((0.0, 0.0, 0.0, 0.0))
        return (r, 0.0) if want_kappa else r
    A = np.ascontiguousarray(Ap)
    n = A.shape[0]
    threads = threads or os.cpu_count() or 1
    out = np.zeros(4)
    ab = np.zeros(1)
    if n == 0:
        r = HighPrec((1.0, 0.0, 0.0, 0.0))
        return (r, 1.0) if want_kappa else r
    rc = _load().orc_formula_range(_dptr(A), n, int(loops), PREC[prec], 1, 1 << (n // 2), threads, _dptr(out),
                                   _dptr(ab))
    if rc != 0:
        raise RuntimeError("oracle formula failed")
    r = HighPrec(out)
    if not want_kappa:
        return r
    mag = abs(r.value)
    return r, (float(ab[0]) / mag if mag else float("inf"))


def formula_masks(A, masks, loops: bool = False, prec: str = "ld", threads: int | None = None) -> HighPrec:
    """Signed sum of f(Z) over an explicit list of subset masks."""
    A = _cplx(A)
    masks = np.ascontiguousarray(np.asarray(masks, dtype=np.uint32))
    out = np.zeros(4)
    threads = threads or os.cpu_count() or 1
    rc = _load().orc_formula_masks(_dptr(A), A.shape[0], int(loops), PREC[prec],
                                   masks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), masks.size, threads,
                                   _dptr(out))
    if rc != 0:
        raise RuntimeError("oracle formula_masks failed")
    return HighPrec(out)


def term(A, mask: int, loops: bool = False, prec: str = "ld") -> HighPrec:
    """One unsigned term f(Z) of the sum, Z given as a bitmask over pairs."""
    A = _cplx(A)
    out = np.zeros(4)
    if _load().orc_term(_dptr(A), A.shape[0], int(loops), PREC[prec], int(mask), _dptr(out)) != 0:
        raise RuntimeError("oracle term failed")
    return HighPrec(out)


def ryser(W, prec: str = "ld", threads: int | None = None) -> HighPrec:
    """Permanent of a square complex matrix (Ryser, Gray-code order)."""
    W = _cplx(W)
    out = np.zeros(4)
    threads = threads or os.cpu_count() or 1
    if _load().orc_ryser(_dptr(W), W.shape[0], PREC[prec], threads, _dptr(out)) != 0:
        raise RuntimeError("oracle ryser failed")
    return HighPrec(out)


# 31-bit primes, all > 2^30 (enough for |value| < 2^(31*k-1) with k primes)
PRIMES = (2147483647, 2147483629, 2147483587, 2147483579, 2147483563, 2147483549, 2147483543)


def modp(A, p: int, loops: bool = False, threads: int | None = None) -> int:
    """haf/lhaf of an integer matrix reduced mod p, via the subset-sum formula."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.int64))
    out = np.zeros(1, dtype=np.uint64)
    threads = threads or os.cpu_count() or 1
    rc = _load().orc_modp(A.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), A.shape[0], int(loops), p, threads,
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if rc != 0:
        raise ValueError("orc_modp: bad arguments")
    return int(out[0])


def modp_term(A, mask: int, p: int, loops: bool = False) -> int:
    A = np.ascontiguousarray(np.asarray(A, dtype=np.int64))
    out = np.zeros(1, dtype=np.uint64)
    rc = _load().orc_modp_term(A.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), A.shape[0], int(loops), p,
                               int(mask), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if rc != 0:
        raise ValueError("orc_modp_term: bad arguments")
    return int(out[0])


def crt(residues, primes):
    """Symmetric-range Chinese remaindering."""
    x, M = 0, 1
    for r, p in zip(residues, primes):
        t = ((r - x) * pow(M, -1, p)) % p
        x += M * t
        M *= p
    if x > M // 2:
        x -= M
    return x, M


def exact_int(A, loops: bool = False, nprimes: int = 5, threads: int | None = None, check: bool = True):
    """Exact integer haf/lhaf of an integer matrix by the formula over several primes.

    With ``check`` one extra prime must agree with the reconstruction.
    Returns (value, seconds).
    """
    A = np.asarray(A, dtype=np.int64)
    n = A.shape[0]
    if n % 2:
        if not loops:
            return 0, 0.0
        B = np.zeros((n + 1, n + 1), dtype=np.int64)
        B[:n, :n] = A
        B[n, n] = 1
        A = B
    t0 = time.time()
    ps = PRIMES[: nprimes + (1 if check else 0)]
    res = [modp(A, p, loops, threads) for p in ps]
    v, _ = crt(res[:nprimes], ps[:nprimes])
    if check and v % ps[-1] != res[-1]:
        raise ArithmeticError("CRT check prime disagrees: value exceeds the prime product")
    return v, time.time() - t0
