"""The C-ABI library loads and exports every function include/hdmr.h declares;
host-side argument checks (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names.update(re.findall(r"^\s*(?:int|void|const char \*)\s*\**\s*(\w+)\s*\(", txt, flags=re.M))
    return sorted(names)


def test_library_exports_header_symbols():
    import paper_2202_06555_amd as hd
    L = hd.lib()
    names = _header_functions()
    assert len(names) >= 9
    for nm in names:
        assert hasattr(L, nm), nm
    assert sorted(hd.EXPORTS) == names


def test_host_validation_errors():
    import paper_2202_06555_amd as hd
    import workloads.synth as ws
    good = ws.synthetic_regular_model(d=3, m=2, order=1, ell=2, seed=0)
    bad = dict(good)
    bad["indices"] = [ix.copy() for ix in good["indices"]]
    bad["indices"][0][0, 0] = 2            # even index violates eq (3.3)
    with pytest.raises(hd.HdmrError) as e:
        hd.hdmr_model_from_surpluses(bad)
    assert e.value.code == hd.hdmr.HDMR_EINVAL
    dup = dict(good)
    dup["levels"] = [np.vstack([lv, lv[:1]]) for lv in good["levels"]]
    dup["indices"] = [np.vstack([ix, ix[:1]]) for ix in good["indices"]]
    dup["alpha"] = [np.vstack([a, a[:1]]) for a in good["alpha"]]
    with pytest.raises(hd.HdmrError) as e:
        hd.hdmr_model_from_surpluses(dup)
    assert "duplicate" in str(e.value)
    big = dict(good)
    big["comps"] = [(0, 1, 2, 0, 1)] + list(good["comps"][1:])
    with pytest.raises(hd.HdmrError) as e:
        hd.hdmr_model_from_surpluses(big)
    assert e.value.code == hd.hdmr.HDMR_EUNSUPPORTED
    assert hd.hdmr_last_error() != ""


def test_timing_switch_without_device():
    import paper_2202_06555_amd as hd
    hd.hdmr_timing_enable(True)
    assert hd.hdmr_timing_read("contract") == (0.0, 0)
    with pytest.raises(hd.HdmrError) as e:
        hd.hdmr_timing_read("nope")
    assert e.value.code == hd.hdmr.HDMR_EINVAL
    hd.hdmr_timing_enable(False)


def test_model_load_rejects_bad_files(tmp_path):
    import paper_2202_06555_amd as hd
    with pytest.raises(hd.HdmrError) as e:
        hd.hdmr_model_load(str(tmp_path / "missing.hdmr"))
    assert e.value.code == hd.hdmr.HDMR_EINVAL
    bad = tmp_path / "bad.hdmr"
    bad.write_bytes(b"not a model file at all")
    with pytest.raises(hd.HdmrError) as e:
        hd.hdmr_model_load(str(bad))
    assert "not a model file" in str(e.value)
    trunc = tmp_path / "trunc.hdmr"
    trunc.write_bytes(b"HDMRASG1" + (1).to_bytes(4, "little") + (4).to_bytes(4, "little"))
    with pytest.raises(hd.HdmrError) as e:
        hd.hdmr_model_load(str(trunc))
    assert e.value.code == hd.hdmr.HDMR_EINVAL


def test_model_load_rejects_oversized_headers(tmp_path):
    # counts in the header or a component header that exceed the file are
    # rejected before any buffer is sized from them (no allocation failure,
    # no exception through the C ABI)
    import struct
    import paper_2202_06555_amd as hd
    head = b"HDMRASG1" + struct.pack("<I", 1)
    cases = {
        "huge_m.hdmr": head + struct.pack("<iii", 4, 2 ** 30, 1) + b"\0" * 64,
        "huge_nc.hdmr": head + struct.pack("<iii", 4, 1, 2 ** 31 - 1) + b"\0" * 64,
        # one component whose row count would overflow n * m in 64 bits
        "huge_rows.hdmr": (head + struct.pack("<iii", 4, 3, 1) + struct.pack("<3d", 0, 0, 0) +
                           struct.pack("<i", 2) + struct.pack("<ii", 0, 1) + struct.pack("<d", 1.0) +
                           struct.pack("<q", 2 ** 62) + b"\0" * 64),
        "negative_rows.hdmr": (head + struct.pack("<iii", 4, 3, 1) + struct.pack("<3d", 0, 0, 0) +
                               struct.pack("<i", 2) + struct.pack("<ii", 0, 1) + struct.pack("<d", 1.0) +
                               struct.pack("<q", -5)),
    }
    for name, data in cases.items():
        f = tmp_path / name
        f.write_bytes(data)
        with pytest.raises(hd.HdmrError) as e:
            hd.hdmr_model_load(str(f))
        assert e.value.code == hd.hdmr.HDMR_EINVAL, name
        assert "corrupt" in str(e.value), name


def test_surrogate_host_validation():
    import paper_2202_06555_amd as hd
    from paper_2202_06555_amd import surrogate as sg
    assert sg.mlp_param_count(300, 512, 151) == 300 * 512 + 512 + 2 * (512 * 512 + 512) + 151 * 512 + 151
    with pytest.raises(hd.HdmrError) as e:
        sg.mlp_param_count(0, 512, 3)
    assert e.value.code == hd.hdmr.HDMR_EINVAL
    with pytest.raises(hd.HdmrError):
        sg.mlp_create(4, 16, 2, np.zeros(5, np.float32))
