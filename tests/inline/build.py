"""Build the on-the-fly consumer (``onthefly.hip``) into ``libonthefly.so``.

It is compiled against the public headers under ``include/`` only, with the
library's own compiler flags, as a user's kernel would be.  Run by path
(``python tests/inline/build.py``) or through ``__graft_entry__.build()``.
"""
import importlib.util
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "onthefly.hip")
LIB = os.path.join(HERE, "libonthefly.so")


def _library_build():
    spec = importlib.util.spec_from_file_location("paper_1101_1846_amd_build",
                                                  os.path.join(ROOT, "paper_1101_1846_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def build():
    B = _library_build()
    flags = [f for f in B.flags() if not f.startswith("-I")] + ["-I" + B.INCLUDE]
    tmp = LIB + ".tmp%d" % os.getpid()
    p = subprocess.run([B.hipcc()] + flags + ["-shared", SRC, "-o", tmp], stdout=subprocess.PIPE,
                       stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("hipcc failed for onthefly.hip:\n" + p.stdout)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
