"""Checkpoint files (paper_1502_07722_amd/checkpoint.py): a host round trip
keeps every bit and the run settings, loads without pickle, refuses other
files; the diagnostics log is one JSON object per line."""
import json

import numpy as np
import pytest

from paper_1502_07722_amd import checkpoint as CK
from paper_1502_07722_amd import workloads as W


def test_round_trip_keeps_bits_and_settings(tmp_path):
    grid, p = W.make_slab(3, (6, 5, 8), 4, 8, 2e-9, 3, fluence_Jcm2=1.0, R_cells=4.0)
    pot = W.hcp(W.morse_cu(c_att=0.3))
    f = tmp_path / "state.npz"
    CK.save_state(f, p, grid, pot, 1e-15, 123, meta={"fluence": 1.0})
    q, g2, pot2, dt, step, meta = CK.load_state(f)
    for a, b in ((p.cell, q.cell), (p.off, q.off), (p.vel, q.vel), (p.wq, q.wq)):
        assert a.dtype == b.dtype and np.array_equal(a.view(np.uint8), b.view(np.uint8))
    assert g2 == grid and pot2 == pot and dt == 1e-15 and step == 123 and meta == {"fluence": 1.0}
    with np.load(f, allow_pickle=False) as z:
        assert set(z.files) == {"cell", "off", "vel", "wq", "header"}
    np.savez(tmp_path / "other.npz", cell=np.zeros(3), header=np.array(json.dumps({"format": "x"})))
    with pytest.raises(ValueError):
        CK.load_state(tmp_path / "other.npz")


def test_diagnostics_log(tmp_path):
    f = tmp_path / "diag.jsonl"
    diags = [{"ke": 1.0, "pe": -2.0, "px": 0.0, "py": 0.0, "pz": 0.0, "wsum": 5.0, "bond": 0.0, "step": 0},
             {"ke": 1.5, "pe": -2.5, "px": 0.0, "py": 0.0, "pz": 0.0, "wsum": 5.0, "bond": 0.0, "step": 1}]
    CK.write_diagnostics(f, diags, step0=100, every=10, meta={"run": "a"})
    lines = [json.loads(x) for x in open(f)]
    assert [x["step"] for x in lines] == [100, 110] and lines[1]["ke"] == 1.5 and lines[0]["run"] == "a"
