"""The C-ABI library loads and exports every entry point include/tpcca.h
declares (no GPU needed), and the binding's struct layouts match the header."""
import ctypes
import os
import re

import numpy as np

from paper_2102_08862_amd import tpcca

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tpcca.h")).read()
    return sorted(set(re.findall(r"\b(tpcca_[a-z_]+)\s*\(", src)))


def test_header_matches_binding_list():
    assert _declared() == sorted(tpcca.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = tpcca.load_library()
    for name in _declared():
        assert hasattr(lib, name), name


def test_struct_layouts(tmp_path):
    """Compile a probe against the header with gcc and compare sizes and
    offsets with the binding's ctypes / numpy layouts."""
    import subprocess
    probe = tmp_path / "probe.c"
    fields = ["frame", "sector", "n_clusters", "status", "first", "seed", "ndf", "x_ref", "y", "t_base", "dt",
              "sinphi", "tau", "qpt", "chi2", "cov"]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "tpcca.h"', 'int main(void){',
             'printf("%zu %zu %zu\\n", sizeof(tpcca_track), sizeof(tpcca_config), sizeof(tpcca_stats));']
    for f in fields:
        lines.append('printf("%%zu\\n", offsetof(tpcca_track, %s));' % f)
    for f, _ in tpcca.Config._fields_:
        lines.append('printf("%%zu\\n", offsetof(tpcca_config, %s));' % f)
    lines.append("return 0;}")
    probe.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I" + os.path.join(ROOT, "include"), str(probe), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    st, sc, ss = int(out[0]), int(out[1]), int(out[2])
    assert st == tpcca.TRACK_DTYPE.itemsize
    assert sc == ctypes.sizeof(tpcca.Config)
    assert ss == ctypes.sizeof(tpcca.Stats)
    offs = [int(v) for v in out[3:]]
    for f, o in zip(fields, offs[: len(fields)]):
        assert tpcca.TRACK_DTYPE.fields[f][1] == o, f
    for (f, _), o in zip(tpcca.Config._fields_, offs[len(fields):]):
        assert getattr(tpcca.Config, f).offset == o, f


def test_default_config_without_gpu():
    c = tpcca.default_config()
    assert abs(c.bz_tesla - 0.5) < 1e-7 and c.n_rows == 152 and c.n_sectors == 36
    x = np.ctypeslib.as_array(c.row_x, shape=(152,))
    assert abs(x[0] - 85.0) < 1e-5 and abs(x[151] - 245.0) < 1e-4
    assert c.kf_passes >= 2 and c.max_gap == 2 and c.min_track_hits == 10
