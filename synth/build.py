"""Build synth/_synthdev.so (device fill of the synthetic B) for gfx950."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = True) -> str:
    src = os.path.join(HERE, "csrc", "synth_fill.hip")
    out = os.path.join(HERE, "_synthdev.so")
    arch = os.environ.get("PNOF_OFFLOAD_ARCH", "gfx950")
    cmd = ["hipcc", f"--offload-arch={arch}", "-O3", "-fPIC", "-shared", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", src, "-o", out + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed:\n{r.stderr}")
    os.replace(out + ".tmp", out)
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    build()
