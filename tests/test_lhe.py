"""LHE 3.0 export from host memory (the writer thread and the record format;
no GPU): events written by lhe_write_events_host read back exactly."""
import math
import os

import numpy as np
import pytest

from oracle import rambo as orb
from lhe_read import read

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2302_03343_amd", "lib",
                   "libvgx.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libvgx.so not built")


def test_host_events_round_trip(tmp_path):
    from paper_2302_03343_amd import vgx
    masses, rs = [173.0, 173.0, 0.0], 1200.0
    k1, w1 = orb.generate(3, 0, 0, 0, 37, masses, rs)
    k2, _ = orb.generate(3, 0, 0, 37, 5, masses, rs)
    path = str(tmp_path / "ev.lhe")
    with vgx.LheWriter(path, beam_energy=(6500.0, 6500.0), xsec=12.5, xsec_err=0.25, xmax=3.0, proc_id=7) as lw:
        lw.write_host(k1, [21, 21], [6, -6, 21], masses, rs, weight=12.5, scale=173.0, aqed=1 / 128, aqcd=0.118,
                      proc_id=7)
        lw.write_host(k2, [21, 21], [6, -6, 21], masses, rs, weight=12.5, scale=173.0, aqed=1 / 128, aqcd=0.118,
                      proc_id=7)
        assert lw.flush() == 42
    root, init, ev = read(path)
    assert root.tag == "LesHouchesEvents" and root.get("version") == "3.0"
    assert [int(v) for v in init[:2]] == [2212, 2212] and float(init[2]) == 6500.0 and int(init[8]) == 3
    assert float(init[10]) == 12.5 and float(init[11]) == 0.25 and float(init[12]) == 3.0 and int(init[13]) == 7
    assert len(ev) == 42
    allk = np.concatenate([k1, k2])
    for e, k in zip(ev, allk):
        assert e["nup"] == 5 and e["proc"] == 7 and e["weight"] == 12.5 and e["aqcd"] == 0.118
        assert e["pdg"] == [21, 21, 6, -6, 21] and e["status"] == [-1, -1, 1, 1, 1]
        assert e["mothers"] == [(0, 0), (0, 0), (1, 2), (1, 2), (1, 2)] and e["spin"] == [9] * 5
        assert np.array_equal(e["p"][2:], k)  # 17 significant digits: exact
        assert np.array_equal(e["p"][0], [rs / 2, 0, 0, rs / 2]) and np.array_equal(e["p"][1], [rs / 2, 0, 0, -rs / 2])
        assert np.array_equal(e["mass"], [0.0, 0.0] + masses)
        assert np.allclose(e["p"][2:].sum(axis=0), e["p"][:2].sum(axis=0), rtol=0, atol=1e-9 * rs)


def test_errors(tmp_path):
    from paper_2302_03343_amd import vgx
    with pytest.raises(vgx.VgxError):
        vgx.LheWriter(str(tmp_path / "no" / "such" / "dir" / "x.lhe"))
    h = vgx.lhe_open(str(tmp_path / "e.lhe"))
    try:
        with pytest.raises(vgx.VgxError):  # more particles than supported
            vgx.lhe_write_events_host(h, np.zeros((1, 11, 4)), [1, 2], list(range(11)), [0.0] * 11, 10.0)
        with pytest.raises(vgx.VgxError):
            vgx.lhe_write_events_host(h, np.zeros((1, 2, 4)), [1, 2], [1, 2], [0.0, 0.0], -1.0)
        with pytest.raises(ValueError):
            vgx.lhe_write_events_host(h, np.zeros((1, 2, 4)), [1, 2], [1, 2, 3], [0.0, 0.0], 10.0)
    finally:
        vgx.lhe_close(h)
    _, _, ev = read(str(tmp_path / "e.lhe"))
    assert ev == []
