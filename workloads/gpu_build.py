"""Build workloads/libmds_gen.so (GPU input generators) for gfx950."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libmds_gen.so")


def build():
    src = os.path.join(HERE, "csrc", "gen.hip")
    tmp = LIB + ".tmp"
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", src, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for gen.hip:\n" + r.stderr)
    os.replace(tmp, LIB)
    print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
