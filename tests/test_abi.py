"""The C ABI library: builds, loads, exports every declared symbol, and its
struct layouts match the header (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mstar.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mstar_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_2001_03180_amd as M
    lib = M.lib()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(M.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", M.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (mstar_\w+)", out))
    assert exported == set(names)


def test_abi_version_and_defaults():
    import paper_2001_03180_amd as M
    lib = M.lib()
    assert lib.mstar_abi_version() == 2
    p = M.params()
    assert p.struct_size == ctypes.sizeof(M.Params)
    assert (p.k_fix, p.n_d, p.eta, p.alpha, p.beta, p.gamma) == (8, 2, 1e-12, 1.0, 0.0, 0.0)
    assert p.accept_rule == 0
    assert lib.mstar_strerror(-6) == b"GBS step did not converge"


def test_struct_layout_matches_header(tmp_path):
    import paper_2001_03180_amd as M
    src = tmp_path / "s.c"
    src.write_text('#include "mstar.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(mstar_params), sizeof(mstar_stats),'
                   ' offsetof(mstar_params, k_fix), offsetof(mstar_stats, t_reached), offsetof(mstar_params, max_steps),'
                   ' offsetof(mstar_params, accept_rule));return 0;}\n')
    exe = tmp_path / "s"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    want = [ctypes.sizeof(M.Params), ctypes.sizeof(M.Stats), M.Params.k_fix.offset, M.Stats.t_reached.offset,
            M.Params.max_steps.offset, M.Params.accept_rule.offset]
    assert [int(g) for g in got] == want


def test_batch_struct_layout_matches_header(tmp_path):
    import numpy as np
    import paper_2001_03180_amd as M
    src = tmp_path / "b.c"
    src.write_text('#include "mstar.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(mstar_batch_stats),'
                   ' offsetof(mstar_batch_stats, steps_accepted), offsetof(mstar_batch_stats, t_reached),'
                   ' sizeof(mstar_batch_config), offsetof(mstar_batch_config, kernel_ms));return 0;}\n')
    exe = tmp_path / "b"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    d = M.BATCH_STATS_DTYPE
    want = [d.itemsize, d.fields["steps_accepted"][1], d.fields["t_reached"][1], ctypes.sizeof(M.BatchConfig),
            M.BatchConfig.kernel_ms.offset]
    assert [int(g) for g in got] == want
    assert np.dtype(d).isalignedstruct or d.itemsize == 88


def test_no_gpu_reports_device_error():
    """Without a GPU, creating a context fails cleanly (no abort across the ABI)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    import paper_2001_03180_amd as M
    h = ctypes.c_void_p()
    assert M.lib().mstar_create(ctypes.byref(h), 0, None) in (M.E_DEVICE, M.E_INVAL)
