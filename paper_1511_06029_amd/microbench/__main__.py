"""Build and run the FP64 matrix-instruction rate probe (one JSON line)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mfma_f64_rate.hip")
EXE = os.path.join(HERE, "_build", "mfma_f64_rate")


def build():
    os.makedirs(os.path.dirname(EXE), exist_ok=True)
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-o", EXE, SRC]
    subprocess.run(cmd, check=True, capture_output=True)


if __name__ == "__main__":
    if not os.path.exists(EXE) or "--build" in sys.argv:
        build()
    if "--build" in sys.argv:
        sys.exit(0)
    sys.exit(subprocess.run([EXE] + [a for a in sys.argv[1:] if a != "--build"]).returncode)
