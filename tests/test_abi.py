"""The C-ABI library loads and exports what include/chimera.h declares; the
binding's struct matches the header (no GPU needed)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "chimera.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(chimera_[a-z0-9_]+)\s*\(", src)))


def test_exports_match_header():
    from paper_2504_02034_amd import chimera
    names = declared()
    assert names and set(names) == set(chimera.EXPORTS)
    for n in names:
        assert hasattr(chimera.lib, n), n


def test_config_layout_matches_header(tmp_path):
    from paper_2504_02034_amd import chimera
    import ctypes
    prog = tmp_path / "cfg.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "chimera.h"\n'
                    'int main(void){printf("%zu %zu %zu %zu\\n", sizeof(chimera_config),'
                    ' offsetof(chimera_config, n_tab), offsetof(chimera_config, device),'
                    ' offsetof(chimera_config, hbm_budget));return 0;}\n')
    exe = tmp_path / "cfg"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    C = chimera.Config
    assert got == [ctypes.sizeof(C), C.n_tab.offset, C.device.offset, C.hbm_budget.offset]


def test_default_config_values():
    from paper_2504_02034_amd import chimera
    c = chimera.chimera_default_config()
    assert (c.n_z, c.z_lo, c.z_hi, c.n_tab, c.z_tab_max) == (1000, 0.0, 1.6, 8192, 25.0)
    assert (c.trunc_fp64, c.trunc_fp32, c.device, c.hbm_budget) == (8.6, 8.6, 0, 0)


def test_bad_config_rejected_without_device():
    from paper_2504_02034_amd import chimera
    c = chimera.chimera_default_config()
    c.n_z = 2
    with pytest.raises(chimera.ChimeraError) as e:
        chimera.chimera_create(c)
    assert e.value.status == chimera.CHIMERA_EINVAL


def test_constants_match_header():
    from paper_2504_02034_amd import chimera
    src = open(os.path.join(ROOT, "include", "chimera.h")).read()
    defined = dict(re.findall(r"#define\s+(CHIMERA_[A-Z_]+)\s+(-?\d+)", src))
    assert int(defined["CHIMERA_MAX_EVENT_PIXELS"]) == chimera.CHIMERA_MAX_EVENT_PIXELS
    assert int(defined["CHIMERA_MAX_BINS"]) == chimera.CHIMERA_MAX_BINS
    enum = dict(re.findall(r"\b(CHIMERA_[A-Z0-9_]+)\s*=\s*(-?\d+)", src))
    for name in ("CHIMERA_OK", "CHIMERA_EINVAL", "CHIMERA_ENOMEM", "CHIMERA_EDEVICE",
                 "CHIMERA_ERANGE", "CHIMERA_ESTATE", "CHIMERA_FP64", "CHIMERA_FP32",
                 "CHIMERA_HOST", "CHIMERA_DEVICE", "CHIMERA_KDE_GAUSSIAN",
                 "CHIMERA_KDE_EPANECHNIKOV"):
        assert int(enum[name]) == getattr(chimera, name), name
