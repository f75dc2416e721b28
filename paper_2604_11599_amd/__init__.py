"""qsv: state-vector execution of OpenQASM 3 dynamic circuits on AMD MI355X.

Front end (host, Python): ``lower`` turns OpenQASM 3 text into the guarded
instruction stream of include/qsv.h. Everything after that — planning, gate
passes, measurement, feed-forward, expectation values, gradients — runs in the
native library libqsv.so (C++ host runtime + gfx950 HIP kernels).
"""
from .frontend import QasmError, parse  # noqa: F401
from .lower import LoweredProgram, lower  # noqa: F401


def __getattr__(name):
    # The GPU binding is imported lazily so that the front end works without the library.
    if name in ("Context", "Program", "QsvError", "plan_inspect"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
