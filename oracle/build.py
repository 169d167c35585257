"""Builds liboracle.so (the FP64 CPU oracle) with gcc.  Test infrastructure."""
import pathlib
import subprocess

HERE = pathlib.Path(__file__).resolve().parent


def build() -> pathlib.Path:
    out = HERE / "liboracle.so"
    tmp = HERE / "liboracle.so.tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-o", str(tmp), str(HERE / "hvpic_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True)
    tmp.replace(out)
    return out


if __name__ == "__main__":
    print(build())
