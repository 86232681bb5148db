"""GPU parity at the benchmark's full size: the 512^3 FP32 Gaussian random field
with a front (seed 2), in the launch configuration bench.py times, against
the oracle on the whole field (streams byte for byte, decompressed values bit
for bit), plus the fault-injected run at eb 1e-4 (6 flips per target on
distinct blocks, counts equal to the oracle's)."""
import numpy as np
import pytest

from oracle import ref
from paper_2010_03144_amd import sdcsz, synth
from tests.gpu_util import first_difference

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPE = (512, 512, 512)
BLOCK = (6, 6, 6)


@pytest.fixture(scope="module")
def field():
    print("generating 512^3 field (seed 2)", flush=True)
    x = synth.grf_field(SHAPE, seed=2)
    return x, torch.from_numpy(x).cuda()


@pytest.fixture(scope="module")
def codec():
    return sdcsz.Codec("cuda:0")


def counts_equal(a, b):
    for t in sdcsz.TARGETS:
        assert a[t] == b[t], (t, a[t], b[t])


@pytest.mark.parametrize("eb,abft", [(1e-3, True), (1e-4, False)])
def test_full_field_identical_to_oracle(codec, field, eb, abft):
    x, xd = field
    print(f"case 512^3 eb={eb} abft={abft}: gpu compress", flush=True)
    rc_g, s_g, rep_g = codec.compress(xd, BLOCK, eb, abft=abft)
    assert rc_g == 0
    s_g_host = s_g.cpu().numpy()
    print("oracle compress", flush=True)
    rc_r, s_r, rep_r = ref.compress(x, BLOCK, eb, abft=abft)
    assert rc_r == 0
    assert np.array_equal(s_r, s_g_host), first_difference(s_r, s_g_host)
    assert rep_r["eb_abs"] == rep_g["eb_abs"]
    print("gpu decompress", flush=True)
    rc, y_g, _ = codec.decompress(s_g)
    assert rc == 0
    y_g = y_g.cpu().numpy()
    print("oracle decompress", flush=True)
    rc, y_r, _ = ref.decompress(s_r)
    assert rc == 0
    assert np.array_equal(y_r.view(np.uint32), y_g.view(np.uint32))
    err = np.abs(x.astype(np.float64) - y_g.astype(np.float64)).max()
    assert err <= rep_g["eb_abs"]


def test_full_field_fault_injection_matches_oracle(codec, field):
    x, xd = field
    counts = {"input": 6, "coef": 6, "code": 6, "dup_pred": 6, "dup_recon": 6}
    plan = synth.fault_plan(SHAPE, BLOCK, np.float32, counts, seed=3)
    print(f"case 512^3 eb=1e-4 fault plan {len(plan)} entries: gpu compress", flush=True)
    rc_g, s_g, rep_g = codec.compress(xd, BLOCK, 1e-4, faults=plan)
    print("oracle compress", flush=True)
    rc_r, s_r, rep_r = ref.compress(x, BLOCK, 1e-4, faults=plan)
    assert rc_r == rc_g == 0
    counts_equal(rep_r, rep_g)
    assert rep_g["generic_plan_blocks"] == 0  # the specialised kernels apply every flip
    for t in ("input", "coef", "code"):
        assert rep_g[t]["injected"] == rep_g[t]["corrected"] == 6, (t, rep_g[t])
    s_g_host = s_g.cpu().numpy()
    assert np.array_equal(s_r, s_g_host), first_difference(s_r, s_g_host)
    # every flip corrected: the stream is the fault-free one
    rc, s_clean, _ = codec.compress(xd, BLOCK, 1e-4)
    assert rc == 0 and np.array_equal(s_clean.cpu().numpy(), s_g_host)
    s_g = torch.from_numpy(s_g_host).cuda()
    # decompression: RECON flips on 6 distinct blocks, re-executed
    rplan = synth.fault_plan(SHAPE, BLOCK, np.float32, {"recon": 6}, seed=33)
    print("gpu decompress with recon faults", flush=True)
    rc_g, y_g, rep_dg = codec.decompress(s_g, faults=rplan)
    print("oracle decompress with recon faults", flush=True)
    rc_r, y_r, rep_dr = ref.decompress(s_r, faults=rplan)
    assert rc_r == rc_g == 0
    counts_equal(rep_dr, rep_dg)
    assert rep_dg["recon"]["detected"] == rep_dg["recon"]["corrected"] == 6
    assert rep_dg["generic_plan_blocks"] == 0
    assert np.array_equal(y_r.view(np.uint32), y_g.cpu().numpy().view(np.uint32))


def test_field_above_2gib_matches_oracle(codec, field):
    """A 2.18 GB FP32 field (1040 x 1024 x 512, mirrored copies of the 512^3
    field): the specialised kernels' wide instantiation (a base per lane
    instead of 32-bit offsets from the wave's lowest block) gives the
    oracle's stream byte for byte and its values bit for bit, and a region
    beyond the first 2 GiB equals the slice of full decompression."""
    x, _ = field
    x2 = np.concatenate([x, x[:, ::-1, :]], axis=1)
    big = np.ascontiguousarray(np.concatenate([x2, x2[::-1], x2[:16]], axis=0))
    del x2
    assert big.nbytes > 2 ** 31
    xd = torch.from_numpy(big).cuda()
    print(f"case {big.shape} ({big.nbytes / 1e9:.2f} GB) eb=1e-3: gpu compress", flush=True)
    rc_g, s_g, rep_g = codec.compress(xd, BLOCK, 1e-3)
    assert rc_g == 0
    s_host = s_g.cpu().numpy()
    print("gpu decompress", flush=True)
    rc, y_g, _ = codec.decompress(s_g)
    assert rc == 0
    lo, hi = (1000, 900, 300), (1040, 1024, 512)
    rc, part, _ = codec.decompress_region(s_g, lo, hi)
    assert rc == 0
    assert torch.equal(part.view(torch.int32), y_g[1000:, 900:, 300:].contiguous().view(torch.int32))
    y_g = y_g.cpu().numpy()
    del xd
    print("oracle compress", flush=True)
    rc_r, s_r, rep_r = ref.compress(big, BLOCK, 1e-3)
    assert rc_r == 0
    assert np.array_equal(s_r, s_host), first_difference(s_r, s_host)
    counts_equal(rep_r, rep_g)
    print("oracle decompress", flush=True)
    rc, y_r, _ = ref.decompress(s_r)
    assert rc == 0
    assert np.array_equal(y_r.view(np.uint32), y_g.view(np.uint32))


def test_wide_2d_fp64_field_round_trip_and_oracle_regions(codec):
    """A 2.15 GB FP64 2D field (16384 x 16400, 16x16 blocks, made on the
    device): the wide 2D kernels keep every value within the bound, and the
    oracle decoding regions of the GPU's stream (at both ends of the field)
    gives the GPU's values bit for bit."""
    g = torch.Generator(device="cuda:0").manual_seed(21)
    xd = torch.randn((16384, 16400), generator=g, device="cuda:0", dtype=torch.float64).cumsum(1).cumsum(0)
    xd = (xd / xd.std()).contiguous()
    assert xd.numel() * 8 > 2 ** 31
    print("case 16384x16400 FP64 eb=1e-4: gpu compress", flush=True)
    rc, s, rep = codec.compress(xd, (16, 16), 1e-4)
    assert rc == 0
    s = s.clone()
    rc, y, _ = codec.decompress(s)
    assert rc == 0
    assert float((xd - y).abs().max()) <= rep["eb_abs"]
    s_host = s.cpu().numpy()
    for lo, hi in (((0, 0), (40, 37)), ((16300, 16350), (16384, 16400)), ((9000, 7000), (9033, 7100))):
        print(f"region {lo} {hi}", flush=True)
        rc_r, part_r, _ = ref.decompress_region(s_host, lo, hi)
        rc_g, part_g, _ = codec.decompress_region(s, lo, hi)
        assert rc_r == rc_g == 0
        assert np.array_equal(part_r.view(np.uint64), part_g.cpu().numpy().view(np.uint64))
        assert torch.equal(part_g.view(torch.int64), y[lo[0]:hi[0], lo[1]:hi[1]].contiguous().view(torch.int64))
