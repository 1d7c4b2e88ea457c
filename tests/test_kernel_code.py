"""Properties of the gfx950 code the HIP sources compile to (no GPU needed):
the reverse-sweep and recording kernels make no device-function calls.

Every adjoint entity function is force-inlined: an out-of-line callee was
once miscompiled (its long-branch expansion used the return-address
registers as scratch without saving them, so a wave that took that branch
returned into the middle of the callee).  Long branches inside a kernel
(s_setpc_b64 to a label of the same kernel) are fine; calls are not."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_04857_amd", "csrc")


def device_asm(source: str, tmp_path) -> str:
    from paper_2506_04857_amd import build
    out = str(tmp_path / (os.path.basename(source) + ".s"))
    flags = [f for f in build.HIPCC_FLAGS if f not in ("-shared",)]
    cmd = [build.hipcc(), *flags, "--cuda-device-only", "-S", "-o", out, os.path.join(CSRC, source)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail("hipcc failed:\n" + r.stderr[-2000:])
    return open(out).read()


def kernels(asm: str):
    """{kernel symbol: its instruction text} for every kernel in the file."""
    out = {}
    for m in re.finditer(r"\n(_Z\w+):\s*;\s*@", asm):
        end = asm.index(".Lfunc_end", m.start())
        out[m.group(1)] = asm[m.start():end]
    return out


def test_adjoint_kernels_make_no_device_calls(tmp_path):
    ks = kernels(device_asm("af_adjoint.hip", tmp_path))
    names = [k for k in ks if re.search(r"k[ar]_(points|limiter|iface|sensor|centre|update)", k)]
    assert len(names) >= 10, names
    for k in names:
        body = ks[k]
        assert "s_swappc_b64" not in body and "s_call_b64" not in body, f"{k} makes a device call"
        # long branches stay inside the kernel
        for tgt in re.findall(r"\((\.LBB\w+)-\.Lpost_getpc\d+\)", body):
            assert tgt + ":" in body, f"{k}: long branch to {tgt} outside the kernel"
