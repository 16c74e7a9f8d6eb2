"""The streaming kernel of the low-bandwidth experiments (Sec. 5): it reads
exactly its share of the buffer, ends at its stop, its wall-clock limit or
its round limit, and a product run beside it keeps its bits and its bound."""
import json
import time

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu
mm = pytest.importorskip("paper_1904_05717_amd")

ROUND = 16384   # bytes one wave reads per round
WAVES = 16      # waves per streamer workgroup


def run_beside(hog, fn, stream):
    hog.start(max_seconds=5.0)
    time.sleep(0.005)   # the streamer is resident before the product is enqueued
    try:
        with torch.cuda.stream(stream):
            hog.mark(stream)
            out = fn()
    finally:
        hog.stop(stream)
    return out, hog.report()


@pytest.mark.parametrize("mode", ["stream", "sleep"])
@pytest.mark.parametrize("member", ["C3C0", "A2C0", "C4A2C0"])
def test_product_beside_the_streamer_keeps_its_bits(member, mode):
    m, n, k = 1536, 1408, 1600
    A, B, C = workloads.gemm_operands(m, n, k)
    dev = torch.device("cuda:0")
    Ad, Bd, Cd = (torch.from_numpy(x).to(dev) for x in (A, B, C))
    hog = mm.BandwidthHog(32, mode=mode, nbytes=1 << 30, device=dev)
    s = hog.concurrent_stream()
    with torch.cuda.stream(s):
        alone = mm.gemm(Ad, Bd, Cd.clone(), alpha=1.0, beta=1.0, member=member)
    s.synchronize()
    beside, rep = run_beside(hog, lambda: mm.gemm(Ad, Bd, Cd.clone(), alpha=1.0, beta=1.0, member=member), s)
    assert torch.equal(alone, beside)
    assert rep["covered"] and not rep["timed_out"] and rep["min_rounds"] > 0, json.dumps(rep)
    assert (rep["bytes"] > 0) == (mode == "stream")
    rows = np.arange(0, m, 97)
    got = beside.cpu().numpy()[rows]
    assert np.all(np.abs(got - oracle.gemm(A[rows], B, C[rows], 1.0, 1.0))
                  <= oracle.error_bound(A[rows], B, C[rows], 1.0, 1.0))


def test_reads_exactly_its_share_and_stops_at_the_round_limit():
    G, rpw, rounds = 8, 70, 64
    nbytes = G * WAVES * ROUND * rpw + 12345     # the ragged tail is never read
    rng = np.random.default_rng(190405722)
    host = rng.integers(0, 256, size=nbytes, dtype=np.uint8)
    hog = mm.BandwidthHog(G, mode="stream", nbytes=nbytes)
    hog.buf.copy_(torch.from_numpy(host))
    hog.start(max_seconds=5.0, max_rounds=rounds)   # no stop: the round limit ends every wave
    rep = hog.report()
    rec = hog.rec.view(-1, 4).cpu().numpy()
    assert np.all(rec[:, 0] == rounds) and not rep["timed_out"]
    assert rep["bytes"] == G * WAVES * rounds * ROUND
    words = host[:G * WAVES * rpw * ROUND].view(np.uint32).reshape(G * WAVES, rpw, ROUND // 4)
    want = np.bitwise_xor.reduce(words[:, :rounds, :].reshape(G * WAVES, -1), axis=1)
    np.testing.assert_array_equal(rec[:, 1].astype(np.uint32), want)


def test_wall_clock_limit_ends_the_control():
    hog = mm.BandwidthHog(16, mode="sleep")
    hog.start(max_seconds=0.05, max_rounds=1 << 20)   # no stop: the clock ends every wave
    rep = hog.report()
    hz = float(mm._lib.momms_lowbw_clock_hz())
    rec = hog.rec.view(-1, 4).cpu().numpy()
    dur = (rec[:, 3] - rec[:, 2]) / hz
    assert rep["timed_out"] and rep["bytes"] == 0
    assert np.all(dur >= 0.05) and np.all(dur < 0.5), (dur.min(), dur.max())


def test_more_workgroups_than_compute_units_is_refused():
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    hog = mm.BandwidthHog(cus + 8, mode="sleep")
    with pytest.raises(ValueError, match="argument 4"):
        hog.start()


def test_a_serialized_stream_pair_is_seen_and_the_hog_still_ends():
    """Work enqueued on the hog's own stream runs only after the hog: the
    report says the product was not covered, and the hog ends at its clock."""
    hog = mm.BandwidthHog(8, mode="sleep")
    hog.start(max_seconds=0.05)
    hog.mark(hog.stream)
    hog.stop(hog.stream)
    rep = hog.report()
    assert rep["timed_out"] and not rep["covered"], json.dumps(rep)
