"""The bounds-checking build of the library (-DGMRES_DEBUG: device checks of
CSR, sliced-ELL, deflation and batched column indices and of the fused slot
ranges; a failed check makes the call return GMRES_EDEVICE) runs the solver
paths -- every Arnoldi variant and SpMV kind, mixed precision, a general
deflation basis, the adjoint, batched, block and adaptive solves -- with no
check failing and the release parity gates met.  The library is loaded in a
child process (tests/debug_build_driver.py) so that this process keeps the
release build.
"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_debug_build_paths_pass_their_checks():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1906_04051_amd import build as B
    if not os.path.exists(B.LIB_DEBUG):
        pytest.fail(f"{B.LIB_DEBUG} is missing: build it with `python -m paper_1906_04051_amd.build`")
    env = dict(os.environ, GMRES_LIB=B.LIB_DEBUG)
    print("child: tests/debug_build_driver.py", flush=True)
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "tests", "debug_build_driver.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    print(r.stdout[-4000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0 and "all cases passed" in r.stdout
