"""The direct global -> LDS loads of the BF16 / FP16 adjoint and Green's
kernels set M0 in inline assembly without declaring it; that is sound only
while the compiled kernels use M0 for nothing else.  Compiles both sources to
AMD assembly for gfx950 (no GPU needed) and checks that every instruction
touching M0 is such a load or its set-up: s_mov_b32 m0, <sgpr>, s_nop 0,
global_load_lds_dwordx4.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2203_05632_amd import build as B

pytestmark = pytest.mark.skipif(shutil.which(B.HIPCC) is None and not os.path.exists(B.HIPCC),
                                reason="hipcc not available")


@pytest.mark.parametrize("src", ["adjoint_lp.hip", "green_lp.hip"])
def test_m0_only_set_for_lds_dma(tmp_path, src):
    out = tmp_path / (src + ".s")
    flags = [f for f in B.FLAGS if f not in ("-fPIC", "-shared")]
    cmd = [B.HIPCC, *flags, "--cuda-device-only", "-S", "-I", os.path.join(B.ROOT, "include"), "-I", B.CSRC,
           "-o", str(out), os.path.join(B.CSRC, src)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    lines = [l.split(";")[0].strip() for l in out.read_text().splitlines()]
    code = [l for l in lines if l and not l.startswith((".", "_")) and not l.endswith(":")]
    uses = [i for i, l in enumerate(code) if re.search(r"\bm0\b", l)]
    dmas = [i for i, l in enumerate(code) if l.startswith("global_load_lds")]
    assert dmas, "no direct LDS loads found"
    assert len(uses) == len(dmas)
    for i in uses:
        assert re.fullmatch(r"s_mov_b32 m0, s\d+", code[i]), code[i]
        assert code[i + 1] == "s_nop 0" and code[i + 2].startswith("global_load_lds_dwordx4"), code[i:i + 3]
