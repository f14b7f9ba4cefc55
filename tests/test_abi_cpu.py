"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every symbol the header declares, its host tables agree with the oracle, and
argument validation returns the documented codes before touching a device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]


@pytest.fixture(scope="module")
def rng():
    import paper_1101_1846_amd as R
    return R


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(rng_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("rng_seed", "rng_generate", "rng_skip", "rng_generate_split", "rng_fused_pi"):
        assert required in names


def test_every_declared_symbol_is_exported(rng):
    out = subprocess.run(["nm", "-D", "--defined-only", rng.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (rng_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        assert hasattr(rng.raw(), n)


def test_host_tables_match_oracle(rng, oracle):
    """The library finds its multipliers with Miller-Rabin; the oracle with
    trial division.  Both must give the paper's 392 and a = 65274."""
    table, n = oracle.mwc16_table()
    assert rng.rng_mwc16_multipliers() == table.tolist()
    assert rng.rng_mwc32_multiplier() == oracle.mwc32_multiplier()


def test_state_words(rng, oracle):
    for name, g in rng.GENERATORS.items():
        assert rng.rng_state_words(g) == oracle.state_words(oracle.GENERATORS[name])


def test_strerror(rng):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert rng.rng_strerror(code)
    assert rng.rng_strerror(-99) == "unknown error"


def test_argument_validation(rng):
    L = rng.raw()
    fake = 0x1000  # never dereferenced: every call below fails validation first
    assert L.rng_generate(99, fake, 1, 1, 0, fake, None) == rng.RNG_EINVAL
    assert L.rng_generate(rng.RNG_XS256, fake, 1, 1, 7, fake, None) == rng.RNG_EINVAL
    assert L.rng_generate(rng.RNG_XS256, None, 1, 1, 0, fake, None) == rng.RNG_EINVAL
    assert L.rng_generate(rng.RNG_XS256, fake, 1, 1, 0, None, None) == rng.RNG_EINVAL
    assert L.rng_generate(rng.RNG_XS256, fake + 2, 1, 1, 0, fake, None) == rng.RNG_EINVAL
    assert L.rng_generate(rng.RNG_XS256, fake, 1 << 40, 1 << 40, 0, fake, None) == rng.RNG_ERANGE
    assert L.rng_generate_ex(rng.RNG_XS256, fake, 1, 1, 0, fake, 96, 8, None) == rng.RNG_EINVAL
    assert L.rng_generate_ex(rng.RNG_XS256, fake, 1, 1, 0, fake, 256, 3, None) == rng.RNG_EINVAL
    # empty work is a no-op that touches nothing
    assert L.rng_generate(rng.RNG_KISS, None, 0, 5, 0, None, None) == rng.RNG_OK
    assert L.rng_generate(rng.RNG_KISS, None, 5, 0, 0, None, None) == rng.RNG_OK
    assert L.rng_seed(0, 1, 0, 4, fake, None) == rng.RNG_EINVAL
    assert L.rng_seed(rng.RNG_MWC32, 1, 0, 4, None, None) == rng.RNG_EINVAL
    assert L.rng_seed(rng.RNG_MWC32, 1, (1 << 64) - 2, 4, fake, None) == rng.RNG_ERANGE
    assert L.rng_skip(rng.RNG_MWC32, None, 4, 5, None) == rng.RNG_EINVAL
    assert L.rng_skip(rng.RNG_MWC32, None, 4, 0, None) == rng.RNG_OK
    assert L.rng_fused_pi(rng.RNG_KISS, fake, 4, 4, fake + 4, None) == rng.RNG_EINVAL
    assert L.rng_set_shape(rng.RNG_XS256, 0, 100, 8) == rng.RNG_EINVAL
    assert L.rng_set_shape(rng.RNG_XS256, 2, 256, 8) == rng.RNG_EINVAL
    assert "generator" in rng.rng_last_error() or rng.rng_last_error()


def test_fold_and_leapfrog_validation(rng):
    L = rng.raw()
    fake = 0x10000
    assert L.rng_generate_fold(99, fake, 4, 4, 0, fake, None) == rng.RNG_EINVAL
    assert L.rng_generate_fold(rng.RNG_XS32, fake, 4, 4, 9, fake, None) == rng.RNG_EINVAL
    assert L.rng_generate_fold(rng.RNG_XS32, None, 4, 4, 0, fake, None) == rng.RNG_EINVAL
    assert L.rng_generate_fold(rng.RNG_XS32, fake, 4, 4, 0, fake + 2, None) == rng.RNG_EINVAL
    assert L.rng_generate_fold(rng.RNG_XS32, None, 4, 0, 0, None, None) == rng.RNG_OK
    for name, g in rng.GENERATORS.items():
        need = rng.rng_leapfrog_workspace_bytes(g, 1 << 10)
        assert need >= (1 << 10) * 4 * rng.rng_state_words(g)
        assert L.rng_generate_leapfrog(g, fake, 1 << 20, 1 << 10, 0, fake, fake, fake, need - 256, None) \
            == rng.RNG_ENOMEM, name
    assert L.rng_generate_leapfrog(rng.RNG_MWC32, fake, 100, 0, 0, fake, fake, fake, 1 << 20, None) \
        == rng.RNG_EINVAL
    assert L.rng_generate_leapfrog(rng.RNG_MWC32, fake, 100, 4, 0, fake, fake, fake + 16, 1 << 20, None) \
        == rng.RNG_EINVAL  # workspace must be 256-byte aligned


def test_calibrate_store_validation(rng):
    L = rng.raw()
    fake = 0x10000
    assert L.rng_calibrate_store(fake, 64, 256, fake, 100, 4, None) == rng.RNG_EINVAL  # workgroup size
    assert L.rng_calibrate_store(fake, 64, 256, fake, 256, 3, None) == rng.RNG_EINVAL  # unroll
    assert L.rng_calibrate_store(None, 64, 256, fake, 256, 4, None) == rng.RNG_EINVAL
    assert L.rng_calibrate_store(fake, 64, 256, fake + 2, 256, 4, None) == rng.RNG_EINVAL
    assert L.rng_calibrate_store(None, 0, 256, None, 256, 4, None) == rng.RNG_OK
    assert L.rng_calibrate_store(fake, 1 << 40, 1 << 40, fake, 256, 4, None) == rng.RNG_ERANGE


def test_shape_roundtrip(rng):
    g, t = rng.RNG_XS32, rng.RNG_F32
    old = rng.rng_get_shape(g, t)
    rng.rng_set_shape(g, t, 512, 4)
    assert rng.rng_get_shape(g, t) == (512, 4)
    rng.rng_set_shape(g, t, *old)


def test_row_shape_classes(rng):
    """Rows of 4 or 8 KiB over whole groups of runs (a multiple of 256
    streams at n = 1024, 128 at 2048) keep a shape of their own; every other
    problem uses rng_set_shape's, and XS256 rows of an odd number of 4 KiB
    outside the run class take at least 512 lanes."""
    L = rng.raw()
    t = rng.RNG_U32
    for name, g in rng.GENERATORS.items():
        main = rng.rng_get_shape(g, t)
        runs = rng.rng_row_shape(g, t, 1 << 20, 1024)
        assert rng.rng_row_shape(g, t, 1 << 19, 2048) == runs
        assert rng.rng_row_shape(g, t, 1 << 20, 256) == main
        assert rng.rng_row_shape(g, t, (1 << 20) + 128, 2048) == runs
        other = rng.rng_row_shape(g, t, (1 << 20) + 64, 1024)   # not a whole number of runs
        if g == rng.RNG_XS256:
            assert other == (max(main[0], 512), main[1])
            assert rng.rng_row_shape(g, t, 4096, 3072) == (max(main[0], 512), main[1])
            assert rng.rng_row_shape(g, t, 4096, 4096) == main
        else:
            assert other == main
        rng.rng_set_row_shape(g, t, 256, 1024, 128, 2)
        assert rng.rng_row_shape(g, t, 1 << 20, 1024) == (128, 2)
        assert rng.rng_get_shape(g, t) == main
        rng.rng_set_row_shape(g, t, 256, 1024, *runs)
        assert rng.rng_row_shape(g, t, 1 << 20, 1024) == runs
    wg, un = ctypes.c_uint32(), ctypes.c_uint32()
    assert L.rng_row_shape(99, t, 256, 1024, ctypes.byref(wg), ctypes.byref(un)) == rng.RNG_EINVAL
    assert L.rng_row_shape(rng.RNG_XS32, 7, 256, 1024, ctypes.byref(wg), ctypes.byref(un)) == rng.RNG_EINVAL
    assert L.rng_row_shape(rng.RNG_XS32, t, 256, 1024, None, None) == rng.RNG_EINVAL
    assert L.rng_set_row_shape(rng.RNG_XS32, t, 256, 1024, 100, 8) == rng.RNG_EINVAL
    assert L.rng_set_row_shape(rng.RNG_XS32, t, 256, 1024, 256, 3) == rng.RNG_EINVAL


def test_split_validation(rng):
    L = rng.raw()
    for name, g in rng.GENERATORS.items():
        assert rng.rng_split_workspace_bytes(g, 1 << 20) == (1 << 20) * 4 * rng.rng_state_words(g)
    fake = 0x10000
    small = ctypes.c_uint64(8)
    assert L.rng_generate_split(rng.RNG_XS256, fake, 1 << 20, 1 << 10, 0, fake, fake, fake, 16, None) \
        == rng.RNG_ENOMEM
    assert L.rng_generate_split(rng.RNG_XS256, fake, 100, 0, 0, fake, fake, fake, 1 << 20, None) \
        == rng.RNG_EINVAL
    assert L.rng_generate_split(rng.RNG_XS256, fake, 100, 4, 0, fake, fake, fake + 4, 1 << 20, None) \
        == rng.RNG_EINVAL
    del small


def test_split_noalloc_validation(rng):
    """The allocation-free split rejects bad arguments, and splits whose thread
    states exceed its scratch array, before any device call."""
    L = rng.raw()
    big = 1 << 40
    assert L.rng_generate_split_noalloc(9, big, 100, 4, 0, big, big, None) == rng.RNG_EINVAL
    assert L.rng_generate_split_noalloc(rng.RNG_MWC32, big, 100, 4, 7, big, big, None) == rng.RNG_EINVAL
    assert L.rng_generate_split_noalloc(rng.RNG_MWC32, None, 100, 4, 0, big, big, None) == rng.RNG_EINVAL
    assert L.rng_generate_split_noalloc(rng.RNG_MWC32, big, 100, 0, 0, big, big, None) == rng.RNG_EINVAL
    assert L.rng_generate_split_noalloc(rng.RNG_MWC32, big, 100, 4, 0, None, big, None) == rng.RNG_EINVAL
    assert L.rng_generate_split_noalloc(rng.RNG_MWC32, big + 2, 100, 4, 0, big, big, None) == rng.RNG_EINVAL
    # XS256: 32 bytes of state per thread, 2^21 threads need 64 MiB > 32 MiB
    assert rng.RNG_SPLIT_NOALLOC_SCRATCH_BYTES == 32 << 20
    assert L.rng_generate_split_noalloc(rng.RNG_XS256, big, 1 << 22, 1 << 21, 0, big, big, None) == rng.RNG_ERANGE
    assert L.rng_generate_split_noalloc(rng.RNG_MWC32, big, 1 << 23, 1 << 23, 0, big, big, None) == rng.RNG_ERANGE
    hdr = open(os.path.join(ROOT, "include", "rng.h")).read()
    assert "#define RNG_SPLIT_NOALLOC_SCRATCH_BYTES (32u << 20)" in hdr


def test_product_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_1101_1846_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "rng_oracle" not in text and "liboracle" not in text, f


def test_inline_consumer_built_on_public_headers():
    """The on-the-fly consumer is built from include/ alone and exports its entry."""
    import ctypes
    here = os.path.dirname(os.path.abspath(__file__))
    lib = os.path.join(here, "inline", "libonthefly.so")
    assert os.path.exists(lib), "tests/inline/libonthefly.so is not built (run __graft_entry__.build())"
    assert hasattr(ctypes.CDLL(lib), "onthefly_draw")
    src = open(os.path.join(here, "inline", "onthefly.hip")).read()
    includes = [l.split()[1] for l in src.splitlines() if l.startswith("#include")]
    assert set(includes) == {"<hip/hip_runtime.h>", "<stdint.h>", '"rng.h"', '"rng_inline.hpp"'}


def test_placement_argument_errors():
    """Argument checks of rng_xs256_placement, taken before any device call."""
    import paper_1101_1846_amd as R
    L = R.raw()
    assert L.rng_xs256_placement(3, None, 1, 1, 0, 16, None, None) == R.RNG_EINVAL
    assert L.rng_xs256_placement(-1, None, 1, 1, 0, 16, None, None) == R.RNG_EINVAL
    assert L.rng_xs256_placement(0, None, 1, 1, 2, 16, None, None) == R.RNG_EINVAL
    assert L.rng_xs256_placement(0, None, 1, 1, 0, None, None, None) == R.RNG_EINVAL
    assert L.rng_xs256_placement(0, None, 1, 1, 0, 16, 16, None) == R.RNG_EINVAL
    assert L.rng_xs256_placement(2, None, 0, 5, 1, None, 16, None) == R.RNG_OK
