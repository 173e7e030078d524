"""Builds of the oracle with one planted mistake, for showing that a pin
catches the mistake it guards (test infrastructure; CPU only).

A mutation is a list of (original text, replacement) pairs applied to the
oracle's C source; each original must occur exactly once, so a mutation
whose anchor has changed fails loudly instead of testing nothing.
"""
from __future__ import annotations

import contextlib
import hashlib
import os
import shutil
import subprocess
import tempfile

import oracle as O

_CACHE = {}


def build(replacements) -> str:
    src = open(O._SRC).read()
    for old, new in replacements:
        n = src.count(old)
        if n != 1:
            raise AssertionError(f"mutation anchor found {n} times (want 1): {old!r}")
        src = src.replace(old, new)
    key = hashlib.sha256(src.encode()).hexdigest()[:16]
    if key in _CACHE and os.path.exists(_CACHE[key]):
        return _CACHE[key]
    d = tempfile.mkdtemp(prefix="orc_mutant_")
    shutil.copy(os.path.join(os.path.dirname(O._SRC), "fslbm_oracle.h"), d)
    c = os.path.join(d, "fslbm_oracle.c")
    with open(c, "w") as fh:
        fh.write(src)
    so = os.path.join(d, f"liboracle_{key}.so")
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-w", c, "-o", so, "-lm"],
                   check=True)
    _CACHE[key] = so
    return so


@contextlib.contextmanager
def planted(replacements):
    """Inside the block, oracle objects are created from the mutated build."""
    so = build(replacements)
    saved = O._lib
    O._lib = O.load(so)
    try:
        yield
    finally:
        O._lib = saved
