"""Build liboracle.so from vmc_oracle.c with gcc (test infrastructure only)."""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build(extra_flags=()):
    src = os.path.join(_HERE, "vmc_oracle.c")
    out = os.path.join(_HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra", "-Werror",
           "-fno-fast-math", "-ffp-contract=off", *extra_flags, src, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
