"""Properties of the built gfx950 code objects (no GPU needed).

Every device helper is inlined into its kernel: the kernels hold no
subroutine calls.  The wave-level helpers (lane shuffles, ballots, DPP scans,
LDS histograms addressed through the wave's LDS window) are written for the
kernel's own context; when the regression threshold scan was compiled as an
out-of-line call, its splits no longer matched the oracle's."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "paper_2605_09950_amd", "csrc", "_build")
LLVM = "/opt/rocm/llvm/bin"
# engine.o holds the host engine and the no-alloc scratch array, no kernels
OBJECTS = {"k_prep.o": True, "k_forest.o": True, "k_importance.o": True, "engine.o": False}


def _tools():
    need = [os.path.join(LLVM, t) for t in ("llvm-objcopy", "clang-offload-bundler",
                                             "llvm-objdump")]
    return need if all(os.path.exists(t) for t in need) else None


@pytest.mark.parametrize("obj", sorted(OBJECTS))
def test_kernels_make_no_device_calls(obj, tmp_path):
    path = os.path.join(BUILD, obj)
    tools = _tools()
    if not os.path.exists(path) or tools is None:
        pytest.skip("built objects or ROCm LLVM tools not present")
    objcopy, bundler, objdump = tools
    fatbin = str(tmp_path / "fatbin")
    code = str(tmp_path / "gfx950.co")
    subprocess.run([objcopy, "--dump-section", f".hip_fatbin={fatbin}", path], check=True,
                   capture_output=True)
    subprocess.run([bundler, "--unbundle", "--type=o",
                    "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--input={fatbin}",
                    f"--output={code}"], check=True, capture_output=True)
    dis = subprocess.run([objdump, "-d", code], check=True, capture_output=True,
                         text=True).stdout
    if OBJECTS[obj]:
        assert "s_endpgm" in dis  # the gfx950 kernels were found
    calls = [ln.strip() for ln in dis.splitlines() if "s_swappc" in ln or "s_setpc" in ln]
    assert not calls, f"{obj}: device subroutine calls {calls[:4]}"
    shutil.rmtree(tmp_path, ignore_errors=True)
