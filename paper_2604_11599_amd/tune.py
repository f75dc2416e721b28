"""Persistence of the plan autotuner's cache (qsv_tune_export / qsv_tune_import).

The library keeps the fastest measured plan options per (device architecture,
qubit count, precision) in memory for the life of the process; these helpers
write that table to a text file and read it back, so a later process loads
programs with tuned plans (Context(..., tuned_plans=True)) without measuring
again.
"""
import ctypes as C
import os

from . import _abi as A
from .api import QsvError


def export_text():
    n = C.c_size_t()
    rc = A.lib().qsv_tune_export(None, 0, C.byref(n))
    if rc:
        raise QsvError(rc, "qsv_tune_export failed")
    buf = C.create_string_buffer(n.value)
    rc = A.lib().qsv_tune_export(buf, n.value, C.byref(n))
    if rc:
        raise QsvError(rc, "qsv_tune_export failed")
    return buf.value.decode()


def import_text(text):
    rc = A.lib().qsv_tune_import(text.encode())
    if rc:
        raise QsvError(rc, "malformed autotuning table")


def save(path):
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    with open(path, "w") as f:
        f.write("# arch n_qubits precision tile_bits low_bits dense_min_cost best_ms default_ms\n")
        f.write(export_text())


def load(path):
    with open(path) as f:
        import_text(f.read())
