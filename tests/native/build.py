"""Build tests/native/libcascade_host.so: the GPU path's per-node arithmetic
(cascade.h) compiled for the host, for CPU unit tests."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
LIB = os.path.join(HERE, "libcascade_host.so")


def build() -> str:
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=off", "-I", os.path.join(ROOT, "paper_1202_6351_amd", "csrc"),
           "-o", LIB + ".tmp", os.path.join(HERE, "cascade_host.hip")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(res.stdout + res.stderr)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build())
