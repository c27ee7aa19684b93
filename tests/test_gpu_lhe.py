"""RAMBO -> unweighting -> asynchronous LHE export on the GPU: the file holds
exactly the kept events, in order, with the device's momenta bit for bit."""
import numpy as np
import pytest

from lhe_read import read

pytestmark = pytest.mark.gpu


def test_generate_unweight_export(vgx, tmp_path):
    import torch
    print("rambo -> unweight -> lhe", flush=True)
    masses, rs = [173.0, 173.0, 4.7, 0.0], 1500.0
    path = str(tmp_path / "events.lhe")
    expect = []
    with vgx.LheWriter(path, xsec=1.0, xmax=1.0) as lw:
        for b, n in enumerate((50_000, 20_000, 120_000)):  # pooled buffer reused, then grown
            mom = torch.empty((4, 4, n), dtype=torch.float64, device="cuda")
            w = torch.empty(n, dtype=torch.float64, device="cuda")
            vgx.rambo_generate(masses, rs, 5, 0, b, 0, mom, w)
            idx = torch.empty(n, dtype=torch.int64, device="cuda")
            k, _ = vgx.unweight(w, 5, 1, b, idx)
            lw.write(mom, idx, k, [21, 21], [6, -6, 5, 21], masses, rs, weight=1.0, scale=173.0)
            expect.append(mom[:, :, idx[:k]].cpu().numpy().transpose(2, 1, 0))
            # the device buffers may be reused once later work is ordered after the call
            mom.fill_(np.nan)
        n_written = lw.flush()
    expect = np.concatenate(expect)
    assert n_written == expect.shape[0] > 1000
    _, _, ev = read(path)
    assert len(ev) == expect.shape[0]
    got = np.stack([e["p"][2:] for e in ev])
    assert np.array_equal(got, expect)
    assert all(e["pdg"] == [21, 21, 6, -6, 5, 21] for e in ev[:10])


def test_export_without_index_list(vgx, tmp_path):
    import torch
    n = 1000
    mom = torch.empty((4, 2, n), dtype=torch.float64, device="cuda")
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    vgx.rambo_generate([0.0, 0.0], 100.0, 1, 0, 0, 0, mom, w)
    path = str(tmp_path / "all.lhe")
    with vgx.LheWriter(path) as lw:
        lw.write(mom, None, 300, [1, -1], [11, -11], [0.0, 0.0], 100.0)
    _, _, ev = read(path)
    ref = mom[:, :, :300].cpu().numpy().transpose(2, 1, 0)
    assert np.array_equal(np.stack([e["p"][2:] for e in ev]), ref)
