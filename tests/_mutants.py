"""Planted mistakes in the oracle, for tests that show a pin catches them.

A mutant is a copy of one oracle function with one textual change: either
the C oracle recompiled from an edited copy of its source (loaded in place
of the real library for the duration of a ``with`` block), or a Python
oracle function re-created from its edited source.  Mutants live only in
the test process; the oracle's files are never touched.
"""
from __future__ import annotations

import contextlib
import ctypes
import inspect
import os
import subprocess

import oracle


def _mutate(src: str, old: str, new: str) -> str:
    if src.count(old) != 1:
        raise AssertionError(f"mutation site must occur exactly once: {old!r}")
    return src.replace(old, new)


@contextlib.contextmanager
def c_oracle_mutant(tmpdir, old: str, new: str):
    """The C oracle built from its source with `old` replaced by `new`."""
    with open(os.path.join(os.path.dirname(oracle.__file__), "ctoracle.c")) as f:
        src = _mutate(f.read(), old, new)
    c = os.path.join(str(tmpdir), "mutant.c")
    so = os.path.join(str(tmpdir), f"mutant{abs(hash(new))}.so")
    with open(c, "w") as f:
        f.write(src)
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE",
                           "-ffp-contract=off", "-o", so, c, "-lm"])
    lib = ctypes.CDLL(so)
    lib.orc_wang_weight.restype = ctypes.c_double
    saved = oracle._L()
    oracle._lib = lib
    try:
        yield lib
    finally:
        oracle._lib = saved


def py_oracle_mutant(fn, old: str, new: str):
    """A copy of the oracle function `fn` with `old` replaced by `new` in its
    source, evaluated in the oracle module's namespace."""
    src = _mutate(inspect.getsource(fn), old, new)
    ns = dict(vars(inspect.getmodule(fn)))
    exec(compile(src, f"<mutant of {fn.__name__}>", "exec"), ns)
    return ns[fn.__name__]
