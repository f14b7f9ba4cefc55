"""Batched path: every request of a batch equals the slice
[offset, offset + length) of its stream's serial sequence (the oracle), its
state ends advanced by offset + length, and results are the same alone and in
the mix, for every launch shape, chunk length and graph replay."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GENS = ["MWC32", "XS256", "XS32", "KISS", "MWC1616"]


@pytest.fixture(scope="module")
def rng():
    import paper_1101_1846_amd as R
    R.rng_init()
    return R


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available()
    return T


def _u32(t):
    import torch as T
    T.cuda.synchronize()
    return t.cpu().numpy().view(np.uint32)


class Mix:
    """A random request mix over per-generator state pools [words][n_g]."""

    def __init__(self, rng, torch, oracle, n, seed, max_len, misalign=True, offsets=True, gens=GENS):
        r = np.random.default_rng(seed)
        self.R, self.T, self.O = rng, torch, oracle
        self.gen = [gens[i] for i in r.integers(0, len(gens), n)]
        self.dtype = r.integers(0, 2, n)
        self.length = r.integers(0, max_len + 1, n)
        self.length[r.random(n) < 0.1] = 0
        self.offset = np.where(r.random(n) < 0.3, r.integers(0, 10 ** 6, n), 0) if offsets else np.zeros(n, int)
        if offsets:
            self.offset[r.random(n) < 0.05] = (1 << 40) + 3
        counts = {g: self.gen.count(g) for g in gens}
        self.pool, self.idx = {}, []
        seen = {g: 0 for g in gens}
        for g in self.gen:
            self.idx.append(seen[g])
            seen[g] += 1
        for g in gens:
            if counts[g]:
                gid = rng.GENERATORS[g]
                st = torch.empty((rng.rng_state_words(gid), counts[g]), dtype=torch.int32, device="cuda")
                rng.rng_seed(gid, 40 + gid, 0, counts[g], st)
                self.pool[g] = st
        self.seed_of = {g: 40 + rng.GENERATORS[g] for g in gens}
        self.counts = counts
        self.offs = []
        pos = 0
        for i in range(n):
            pos = (pos + 3) // 4 * 4 + (int(r.integers(0, 4)) if misalign else 0)
            self.offs.append(pos)
            pos += int(self.length[i])
        self.out = torch.zeros(pos + 8, dtype=torch.int32, device="cuda")

    def requests(self, subset=None):
        R = self.R
        reqs = []
        for i in (range(len(self.gen)) if subset is None else subset):
            g = self.gen[i]
            pool = self.pool[g]
            base = pool.data_ptr() + 4 * self.idx[i]
            reqs.append((R.GENERATORS[g], int(self.dtype[i]), base, self.counts[g], int(self.offset[i]),
                         int(self.length[i]), self.out.data_ptr() + 4 * self.offs[i]))
        return reqs

    def expected(self, i, pass_no=1):
        """Oracle output of request i on its `pass_no`-th run from the seeded pool."""
        O, g = self.O, self.gen[i]
        o = O.GENERATORS[g]
        st = O.seed(o, self.seed_of[g], 1, first_stream=self.idx[i])
        out = None
        for _ in range(pass_no):
            if self.offset[i]:
                O.skip(o, st, int(self.offset[i]))
            out = O.generate(o, st, int(self.length[i]), int(self.dtype[i]))[0]
        return out.view(np.uint32), st[:, 0]

    def check(self, subset=None, pass_no=1):
        got = _u32(self.out)
        pools = {g: _u32(p) for g, p in self.pool.items()}
        for i in (range(len(self.gen)) if subset is None else subset):
            exp, st = self.expected(i, pass_no)
            n = int(self.length[i])
            assert np.array_equal(got[self.offs[i]:self.offs[i] + n], exp), (i, self.gen[i], n)
            assert np.array_equal(pools[self.gen[i]][:, self.idx[i]], st), (i, "state")


def test_batch_mixed_requests(rng, torch, oracle):
    m = Mix(rng, torch, oracle, 300, seed=1, max_len=20000)
    h = rng.rng_batch_create(1000, 1 << 24)
    try:
        rng.rng_batch_set(h, m.requests())
        rng.rng_batch_launch(h)
        m.check()
    finally:
        rng.rng_batch_destroy(h)


def test_batch_alone_equals_in_mix(rng, torch, oracle):
    mix = Mix(rng, torch, oracle, 120, seed=2, max_len=9000)
    alone = Mix(rng, torch, oracle, 120, seed=2, max_len=9000)
    h = rng.rng_batch_create(200, 1 << 22)
    try:
        rng.rng_batch_set(h, mix.requests())
        rng.rng_batch_launch(h)
        for i in (0, 7, 33, 119):
            rng.rng_batch_set(h, alone.requests([i]))
            rng.rng_batch_launch(h)
        torch.cuda.synchronize()
        a, b = _u32(mix.out), _u32(alone.out)
        for i in (0, 7, 33, 119):
            n = int(mix.length[i])
            assert np.array_equal(a[mix.offs[i]:mix.offs[i] + n], b[alone.offs[i]:alone.offs[i] + n])
        alone.check([0, 7, 33, 119])
    finally:
        rng.rng_batch_destroy(h)


@pytest.mark.parametrize("shape", [(wg, u) for wg in (64, 128, 256, 512, 1024) for u in (1, 2, 4, 8, 16)])
def test_batch_every_shape(rng, torch, oracle, shape):
    m = Mix(rng, torch, oracle, 80, seed=3, max_len=6000)
    h = rng.rng_batch_create(100, 1 << 20)
    try:
        rng.rng_batch_set_shape(h, shape[0], shape[1], 0)
        assert rng.rng_batch_get_shape(h)[:2] == shape
        rng.rng_batch_set(h, m.requests())
        rng.rng_batch_launch(h)
        m.check()
    finally:
        rng.rng_batch_destroy(h)


@pytest.mark.parametrize("chunk", [64, 192, 1024, 4096])
def test_batch_chunk_lengths(rng, torch, oracle, chunk):
    m = Mix(rng, torch, oracle, 60, seed=4, max_len=30000)
    h = rng.rng_batch_create(100, 1 << 22)
    try:
        rng.rng_batch_set_shape(h, 0, 0, chunk)
        rng.rng_batch_set(h, m.requests())
        rng.rng_batch_launch(h)
        m.check()
    finally:
        rng.rng_batch_destroy(h)


def test_batch_tree_path(rng, torch, oracle):
    """More than 2^15 chunks (64-sample chunks over about 3e6 samples): the chunk
    start states come from the doubling tree rather than direct jumps."""
    m = Mix(rng, torch, oracle, 300, seed=5, max_len=20000)
    assert sum(-(-int(n) // 64) for n in m.length) > (1 << 15)
    h = rng.rng_batch_create(1000, 1 << 24)
    try:
        rng.rng_batch_set_shape(h, 0, 0, 64)
        rng.rng_batch_set(h, m.requests())
        rng.rng_batch_launch(h)
        m.check()
    finally:
        rng.rng_batch_destroy(h)


@pytest.mark.parametrize("n,max_len", [(1, 1 << 17), (5, 1 << 20), (300, 20000)])
def test_batch_auto_chunk(rng, torch, oracle, n, max_len):
    """Automatic chunk length: every plan picks C from the batch's size."""
    m = Mix(rng, torch, oracle, n, seed=6 + n, max_len=max_len)
    h = rng.rng_batch_create(1000, 1 << 24)
    try:
        rng.rng_batch_set_shape(h, 0, 0, rng.RNG_BATCH_CHUNK_AUTO)
        assert rng.rng_batch_get_shape(h)[2] == rng.RNG_BATCH_CHUNK_AUTO
        rng.rng_batch_set(h, m.requests())
        rng.rng_batch_launch(h)
        m.check()
    finally:
        rng.rng_batch_destroy(h)


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_graph_replays(rng, torch, oracle, use_graph):
    """The same plan launched three times, with eager library work and a
    synchronisation between replays: replay k must give pass k of every stream
    (kernels launched directly, and replayed from the captured graph)."""
    m = Mix(rng, torch, oracle, 50, seed=5, max_len=5000, offsets=False)
    h = rng.rng_batch_create(64, 1 << 20)
    rng.rng_batch_set_graph(h, use_graph)
    side = torch.empty((1, 4096), dtype=torch.int32, device="cuda")
    side_out = torch.empty(4096 * 64, dtype=torch.int32, device="cuda")
    try:
        rng.rng_batch_set(h, m.requests())
        for k in (1, 2, 3):
            rng.rng_batch_launch(h)
            torch.cuda.synchronize()
            m.check(pass_no=k)
            rng.rng_seed(rng.RNG_XS32, 9, 0, 4096, side)
            rng.rng_generate(rng.RNG_XS32, side, 4096, 64, 0, side_out)
            torch.cuda.synchronize()
            rng.rng_batch_set(h, m.requests())
    finally:
        rng.rng_batch_destroy(h)


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_plans_of_different_sizes(rng, torch, oracle, use_graph):
    """Plans of very different sizes on one handle (different tree depths and
    tile counts): a one-request plan, a 200-request plan with long requests,
    then the small one again.  Each run is checked against the oracle's pass
    over those streams."""
    m = Mix(rng, torch, oracle, 200, seed=31, max_len=60000, offsets=False)
    h = rng.rng_batch_create(256, 1 << 24)
    rng.rng_batch_set_graph(h, use_graph)
    try:
        rng.rng_batch_set_shape(h, 0, 0, 64)  # many chunks per request: several tree levels
        runs = {i: 0 for i in range(200)}
        for subset in ([7], list(range(200)), [7]):
            rng.rng_batch_set(h, m.requests(subset))
            rng.rng_batch_launch(h)
            torch.cuda.synchronize()
            for i in subset:
                runs[i] += 1
            got = _u32(m.out)
            pools = {g: _u32(p) for g, p in m.pool.items()}
            for i in subset:
                exp, st = m.expected(i, runs[i])
                n = int(m.length[i])
                assert np.array_equal(got[m.offs[i]:m.offs[i] + n], exp), (subset[:3], i)
                assert np.array_equal(pools[m.gen[i]][:, m.idx[i]], st), (i, "state")
    finally:
        rng.rng_batch_destroy(h)


def test_batch_small_plans_back_to_back(rng, torch, oracle):
    """Small plans travel in the root kernel's arguments, and the root kernel
    writes them to the device plan buffer for the kernels after it: four
    one- and two-request plans launched back to back on one stream with no
    synchronisation in between, then every output checked."""
    m = Mix(rng, torch, oracle, 12, seed=37, max_len=40000, offsets=False)
    h = rng.rng_batch_create(16, 1 << 20)
    try:
        rng.rng_batch_set_shape(h, 0, 0, 64)
        subsets = ([3], [5, 8], [11], [0, 3])
        runs = {i: 0 for i in range(12)}
        for subset in subsets:
            rng.rng_batch_set(h, m.requests(subset))
            rng.rng_batch_launch(h)
            for i in subset:
                runs[i] += 1
        torch.cuda.synchronize()
        got = _u32(m.out)
        pools = {g: _u32(p) for g, p in m.pool.items()}
        for i in {i for sub in subsets for i in sub}:
            exp, st = m.expected(i, runs[i])
            n = int(m.length[i])
            assert np.array_equal(got[m.offs[i]:m.offs[i] + n], exp), i
            assert np.array_equal(pools[m.gen[i]][:, m.idx[i]], st), (i, "state")
    finally:
        rng.rng_batch_destroy(h)


@pytest.mark.parametrize("chunk", [64, 192])
@pytest.mark.parametrize("name", GENS)
def test_batch_small_tree(rng, torch, oracle, chunk, name):
    """Small plans (at most 16^3 chunks per request, in the kernel's
    arguments) build every request's radix-16 tree in one launch (four
    workgroups per request, which share level 2): one request per batch with 1, 15, 16, 17, 255, 256, 257, 1000, 2049 and 4096
    chunks, then all ten in one batch, some with an offset; 64-sample chunks
    (XS256 from LDS-staged tables, level 2 four lanes per source chunk) and
    192 (no power of two: the global digit tables).  Every sample and every
    final state against the oracle."""
    g, o = rng.GENERATORS[name], oracle.GENERATORS[name]
    counts = [1, 15, 16, 17, 255, 256, 257, 1000, 2049, 4096]
    lengths = [c * chunk - (chunk // 2 if c > 1 else 0) for c in counts]
    offsets = [0, 0, 12345, 0, 0, 999, 0, 5, 0, (1 << 33) + 7]
    n = len(counts)
    W = rng.rng_state_words(g)
    st = torch.empty((W, n), dtype=torch.int32, device="cuda")
    rng.rng_seed(g, 71, 0, n, st)
    offs, pos = [], 0
    for L in lengths:
        offs.append(pos)
        pos += (L + 31) // 32 * 32
    out = torch.zeros(pos, dtype=torch.int32, device="cuda")
    ref_st = oracle.seed(o, 71, n)
    h = rng.rng_batch_create(16, 1 << 22)
    try:
        rng.rng_batch_set_shape(h, 0, 0, chunk)
        for subset in [[i] for i in range(n)] + [list(range(n))]:
            reqs = [(g, 0, st.data_ptr() + 4 * i, n, offsets[i], lengths[i], out.data_ptr() + 4 * offs[i])
                    for i in subset]
            rng.rng_batch_set(h, reqs)
            rng.rng_batch_launch(h)
            torch.cuda.synchronize()
            got = _u32(out)
            for i in subset:
                one = ref_st[:, i:i + 1].copy()
                if offsets[i]:
                    oracle.skip(o, one, offsets[i])
                exp = oracle.generate(o, one, lengths[i])[0].view(np.uint32)
                ref_st[:, i] = one[:, 0]
                assert np.array_equal(got[offs[i]:offs[i] + lengths[i]], exp), (subset, i)
            assert np.array_equal(_u32(st), ref_st), subset
    finally:
        rng.rng_batch_destroy(h)


def test_batch_validation(rng, torch):
    h = rng.rng_batch_create(4, 1000)
    st = torch.empty(8, dtype=torch.int32, device="cuda")
    out = torch.empty(2000, dtype=torch.int32, device="cuda")
    try:
        import ctypes
        L = rng.raw()
        bad = [
            [(99, 0, st, 1, 0, 10, out)],
            [(rng.RNG_XS32, 5, st, 1, 0, 10, out)],
            [(rng.RNG_XS32, 0, 0, 1, 0, 10, out)],
            [(rng.RNG_XS32, 0, st, 0, 0, 10, out)],
            [(rng.RNG_XS32, 0, st, 1, 0, 10, out.data_ptr() + 2)],
        ]
        for b in bad:
            arr = rng.make_requests(b)
            assert L.rng_batch_set(h, arr, 1) == rng.RNG_EINVAL
        shared = rng.make_requests([(rng.RNG_XS32, 0, st, 1, 0, 10, out),
                                    (rng.RNG_XS32, 0, st, 1, 5, 10, out.data_ptr() + 64)])
        assert L.rng_batch_set(h, shared, 2) == rng.RNG_EINVAL  # one state, two requests
        distinct = rng.make_requests([(rng.RNG_XS32, 0, st, 1, 0, 10, out),
                                      (rng.RNG_XS32, 0, st.data_ptr() + 4, 1, 5, 10, out.data_ptr() + 64)])
        assert L.rng_batch_set(h, distinct, 2) == rng.RNG_OK
        too_many = rng.make_requests([(rng.RNG_XS32, 0, st, 1, 0, 1, out)] * 5)
        assert L.rng_batch_set(h, too_many, 5) == rng.RNG_ENOMEM
        too_long = rng.make_requests([(rng.RNG_XS32, 0, st, 1, 0, 1001, out)])
        assert L.rng_batch_set(h, too_long, 1) == rng.RNG_ENOMEM
        assert L.rng_batch_set_shape(h, 96, 8, 0) == rng.RNG_EINVAL
        assert L.rng_batch_set_graph(h, 2) == rng.RNG_EINVAL
        assert L.rng_batch_set_shape(h, 256, 8, 100) == rng.RNG_EINVAL
        del ctypes
    finally:
        rng.rng_batch_destroy(h)


def test_batch_empty_and_skip_only(rng, torch, oracle):
    """A batch of zero-length requests only advances the states by their offsets."""
    st = torch.empty((8, 3), dtype=torch.int32, device="cuda")
    rng.rng_seed(rng.RNG_XS256, 11, 0, 3, st)
    h = rng.rng_batch_create(8, 100)
    try:
        reqs = [(rng.RNG_XS256, 0, st.data_ptr() + 4 * i, 3, 1000 * (i + 1), 0, 0) for i in range(3)]
        rng.rng_batch_set(h, reqs)
        rng.rng_batch_launch(h)
        ref = oracle.seed(oracle.XS256, 11, 3)
        for i in range(3):
            col = np.ascontiguousarray(ref[:, i:i + 1])
            oracle.skip(oracle.XS256, col, 1000 * (i + 1))
            assert np.array_equal(_u32(st)[:, i], col[:, 0])
        rng.rng_batch_set(h, [])
        rng.rng_batch_launch(h)
        torch.cuda.synchronize()
    finally:
        rng.rng_batch_destroy(h)
