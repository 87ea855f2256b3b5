"""The ctypes structures of the binding have the C header's layout: a small C
program built with gcc against include/qap_rlt2.h prints every struct's size
and each field's offset, and they must equal ctypes' (CPU only)."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

from paper_1710_03732_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PAIRS = [
    (B.QapParams, "qap_params"), (B.QapDaStats, "qap_da_stats"), (B.QapSaParams, "qap_sa_params"),
    (B.QapBnbParams, "qap_bnb_params"), (B.QapBnbStats, "qap_bnb_stats"), (B.QapBatchParams, "qap_batch_params"),
    (B.QapBatchStats, "qap_batch_stats"), (B.QapStateHeader, "qap_state_header"),
    (B.QapAdamParams, "qap_adam_params"), (B.QapWarmStats, "qap_warm_stats"),
]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_struct_layouts_match_header(tmp_path):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "qap_rlt2.h"', "int main(void) {"]
    for cls, name in PAIRS:
        lines.append(f'    printf("{name} %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            lines.append(f'    printf("{name}.{f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = dict(line.split() for line in out if line)
    for cls, name in PAIRS:
        assert int(got[name]) == C.sizeof(cls), name
        for f in cls._fields_:
            assert int(got[f"{name}.{f[0]}"]) == getattr(cls, f[0]).offset, (name, f[0])
