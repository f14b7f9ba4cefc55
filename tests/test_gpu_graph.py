"""Entry points captured into a HIP graph (through torch's graph capture) after
rng_init(): every replay must continue the streams exactly, with eager work
and synchronisations between the replays.  Covers the resident schedule
(whole stream groups), the chunked path (few streams, jumps inside the
kernel), skip, split and the fused consumer."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

REPLAYS = 3


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


def _eager_noise(torch):
    a = torch.randn(1 << 20, device="cuda")
    (a * 2 + 1).sum().item()


@pytest.mark.parametrize("name,S,N,dt", [("XS256", (1 << 17) + 64, 256, "u32"), ("KISS", (1 << 17) + 64, 128, "f32"),
                                         ("MWC32", 64, 4096, "u32"), ("MWC1616", 3, 5000, "f32")])
def test_generate_graph_replays(rng, torch, oracle, name, S, N, dt):
    g, o, t = rng.GENERATORS[name], oracle.GENERATORS[name], rng.DTYPES[dt]
    st = torch.empty((rng.rng_state_words(g), S), dtype=torch.int32, device="cuda")
    rng.rng_seed(g, 51, 0, S, st)
    out = torch.empty(S * N, dtype=torch.int32, device="cuda")
    rng.rng_generate(g, st, S, N, t, out)  # first call outside the graph (shape choice, occupancy query)
    torch.cuda.synchronize()
    ref_st = oracle.seed(o, 51, S)
    first = oracle.generate(o, ref_st, N, t, threads=8)
    assert np.array_equal(_u32(out).reshape(S, N), first.view(np.uint32))
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        rng.rng_generate(g, st, S, N, t, out)
    for _ in range(REPLAYS):
        _eager_noise(torch)
        graph.replay()
        torch.cuda.synchronize()
        exp = oracle.generate(o, ref_st, N, t, threads=8)
        assert np.array_equal(_u32(out).reshape(S, N), exp.view(np.uint32))
        assert np.array_equal(_u32(st), ref_st)


def test_skip_and_fused_graph_replays(rng, torch, oracle):
    g, o, S, N = rng.RNG_KISS, oracle.KISS, 1000, 2000
    st = torch.empty((6, S), dtype=torch.int32, device="cuda")
    rng.rng_seed(g, 52, 0, S, st)
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        rng.rng_skip(g, st, S, 12345)
        rng.rng_fused_pi(g, st, S, N, cnt)
    ref_st = oracle.seed(o, 52, S)
    total = 0
    for _ in range(REPLAYS):
        _eager_noise(torch)
        graph.replay()
        torch.cuda.synchronize()
        oracle.skip(o, ref_st, 12345)
        total += oracle.fused_pi(o, ref_st, N)
        assert int(cnt.item()) == total
        assert np.array_equal(_u32(st), ref_st)


def test_split_graph_replays(rng, torch, oracle):
    g, o, total, T = rng.RNG_XS256, oracle.XS256, 100000, 1000
    s1 = torch.empty(8, dtype=torch.int32, device="cuda")
    rng.rng_seed(g, 53, 0, 1, s1)
    wsb = rng.rng_split_workspace_bytes(g, T)
    ws = torch.empty(wsb // 4 + 64, dtype=torch.int32, device="cuda")
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    rng.rng_generate_split(g, s1, total, T, rng.RNG_U32, out, s1, ws, wsb)  # once outside the capture
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        rng.rng_generate_split(g, s1, total, T, rng.RNG_U32, out, s1, ws, wsb)  # advances s1 in place
    one = oracle.seed(o, 53, 1)
    oracle.generate(o, one, total)
    for _ in range(REPLAYS):
        _eager_noise(torch)
        graph.replay()
        torch.cuda.synchronize()
        exp = oracle.generate(o, one, total)[0]
        assert np.array_equal(_u32(out), exp)
        assert np.array_equal(_u32(s1), one[:, 0])
