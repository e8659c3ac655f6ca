"""The C-ABI library loads and exports every entry point of include/lbpc.h
(no compute call, no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lbpc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbpc_[a-z_A-Z0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libpath():
    from paper_1703_02652_amd._lib import LIB_PATH
    if not os.path.exists(LIB_PATH):
        from paper_1703_02652_amd.build import build
        build()
    return LIB_PATH


def test_library_exports_every_declared_symbol(libpath):
    lib = ctypes.CDLL(libpath)
    declared = _declared()
    assert len(declared) >= 20
    missing = [s for s in declared if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_covers_header(libpath):
    from paper_1703_02652_amd import EXPORTS
    assert sorted(EXPORTS) == _declared()


def test_version_and_validation_without_gpu(libpath):
    """Calls that touch no device: version string and config validation."""
    import workloads as W
    from paper_1703_02652_amd import lib
    from paper_1703_02652_amd._lib import make_configs
    L = lib()
    assert b"gfx950" in L.lbpc_version()
    good = W.cavity_128()
    assert L.lbpc_workspace_bytes(make_configs([good]), 1) > 2 * 104 * 128**3
    bad = dict(good, face_bc=[0, 1, 2, 2, 2, 2])
    assert L.lbpc_workspace_bytes(make_configs([bad]), 1) == 0
    assert b"periodic" in L.lbpc_last_error(None)
    bad = dict(good, omega_T=0.5)
    assert L.lbpc_workspace_bytes(make_configs([bad]), 1) == 0
    bad = dict(good, s_e=2.5)
    assert L.lbpc_workspace_bytes(make_configs([bad]), 1) == 0
    mixed = [good, dict(good, precision=W.FP64)]
    assert L.lbpc_workspace_bytes(make_configs(mixed), 2) == 0
    assert L.lbpc_workspace_bytes(make_configs([good]), 0) == 0    # empty batch
    assert L.lbpc_workspace_bytes(None, 1) == 0
    # 32-bit byte offsets of 8-byte elements bound a cavity to 2^29 cells
    assert L.lbpc_workspace_bytes(make_configs([dict(good, nx=812, ny=812, nz=812)]), 1) > 0
    assert L.lbpc_workspace_bytes(make_configs([dict(good, nx=813, ny=813, nz=813)]), 1) == 0
    assert b"2^29" in L.lbpc_last_error(None)


def test_config_struct_layout_matches_header():
    """The ctypes mirror has the field order and size of lbpc_config."""
    from paper_1703_02652_amd import LbpcConfig
    text = open(os.path.join(ROOT, "include", "lbpc.h")).read()
    body = text[text.index("typedef struct lbpc_config"):text.index("} lbpc_config;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"\b([a-zA-Z_][a-zA-Z_0-9]*)\s*(?:\[\d+\])?\s*[,;]", body)
    assert names == [n for n, _ in LbpcConfig._fields_]
    assert ctypes.sizeof(LbpcConfig) == 6 * 4 + 6 * 4 + 6 * 8 + 17 * 8 + 7 * 8 + 8


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus 2 exits with status 2 and says why,
    before touching any device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
