"""Build the test-only input kernel of the travelling manufactured solutions
(tests/mms_input_kernel.hip -> tests/libmmsinput.so) with hipcc for gfx950."""
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libmmsinput.so")


def build() -> str:
    cc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([cc, "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-o", tmp, os.path.join(HERE, "mms_input_kernel.hip")])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
