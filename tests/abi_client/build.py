"""Build the C client of the library (tests/abi_client/abi_client.c) with gcc.

The client links libspc3d.so, the oracle's liboracle.so and the HIP runtime;
run-time paths point at the in-tree libraries relative to the binary, so the
tree can move.  Called by the repository's build entry point after the
libraries are built."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
BIN = os.path.join(HERE, "abi_client")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build() -> str:
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           os.path.join(HERE, "abi_client.c"),
           "-L", os.path.join(ROOT, "paper_2404_19638_amd"), "-lspc3d",
           "-L", os.path.join(ROOT, "oracle"), "-loracle",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lm",
           "-Wl,-rpath,$ORIGIN/../../paper_2404_19638_amd:$ORIGIN/../../oracle:" +
           os.path.join(ROCM, "lib"),
           "-o", BIN + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(BIN + ".tmp", BIN)
    return BIN


if __name__ == "__main__":
    print(build())
