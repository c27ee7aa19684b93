"""The C-ABI library loads and exports every entry point the header declares
(no GPU needed: nothing is called that touches a device)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vgx.h")
LIB = os.path.join(ROOT, "paper_2302_03343_amd", "lib", "libvgx.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "for", "return")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("vegas_create", "vegas_iterate", "vegas_refine", "pdf_interp", "flow_sample", "flow_train_step",
                 "batch_iterate", "vgx_last_error"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvgx.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    # loaded through the binding, which loads PyTorch's HIP runtime first
    from paper_2302_03343_amd import vgx
    lib = vgx._lib
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvgx.so not built")
def test_exports_nothing_else():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = sorted(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert exported == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvgx.so not built")
def test_binding_has_the_same_names():
    import paper_2302_03343_amd.vgx as vgx
    for n in declared_functions():
        if n in ("vgx_last_error", "vgx_version"):
            continue
        assert hasattr(vgx, n), n
    assert vgx.version().startswith("vgx")


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvgx.so not built")
@pytest.mark.parametrize("dim", [2, 3, 5, 8, 12])
def test_flow_layout_matches_oracle_on_host(dim):
    # host-only entry point: segment list equals the oracle's reading of the masks
    import paper_2302_03343_amd.vgx as vgx
    from oracle import flow
    assert vgx.flow_param_layout(dim) == flow.init_segments(dim, 4, 32, 64)
    assert vgx.flow_num_params(dim, 4, 32, 64) == flow.n_params(dim, 4, 32, 64)
