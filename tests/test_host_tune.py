"""Host-only parts of the plan autotuner: the cache's text form (import,
export, validation). No device calls."""
import pytest


def test_tune_table_round_trip_and_validation():
    from paper_2604_11599_amd import QsvError, tune
    tune.import_text("# comment\ngfx000 9 c128 11 5 0 1.25 2.5\ngfx000 9 c64 10 4 3 0.5 0.75\n")
    text = tune.export_text()
    assert "gfx000 9 c128 11 5 0 1.25 2.5\n" in text
    assert "gfx000 9 c64 10 4 3 0.5 0.75\n" in text
    tune.import_text("gfx000 9 c128 12 4 0.5 1 1\n")          # later entries replace equal keys
    assert "gfx000 9 c128 12 4 0.5 1 1\n" in tune.export_text()
    for bad in ("gfx000 9 c32 11 5 0 1 1\n", "gfx000 40 c128 11 5 0 1 1\n", "gfx000 9 c128 13 4 0 1 1\n",
                "gfx000 9 c128 11 12 0 1 1\n", "gfx000 9 c128 11 5 -1 1 1\n", "gfx000 9 c128 11\n"):
        with pytest.raises(QsvError):
            tune.import_text(bad)
    assert "gfx000 9 c128 12 4 0.5 1 1\n" in tune.export_text()  # nothing added by a rejected table
