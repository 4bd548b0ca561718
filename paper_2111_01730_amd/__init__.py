"""hodbf: MI355X-native HOD-BF compressed VIE operator, approximate inverse and FGMRES.

The compute lives in ``libhodbf.so`` (hand-written HIP for gfx950 behind a C ABI,
declared in ``include/hodbf.h``); this package only marshals arguments.
"""
from ._lib import HodbfError, lib  # noqa: F401

__all__ = ["HodbfError", "lib", "Operator"]


def __getattr__(name):
    if name == "Operator":
        from .hodbf import Operator
        return Operator
    raise AttributeError(name)
