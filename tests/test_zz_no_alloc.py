"""GPU test of tt_channel_apply_ul_noalloc, the UL call that allocates
nothing: on two channels set up alike, its outputs equal tt_channel_apply_ul's
bit for bit over two calls in a row (the second shorter and with fewer UEs,
so the device scratch holds the first call's partials when the second
starts), free device memory does not change across its calls, and a call
whose partials exceed the scratch is refused before any work."""
import numpy as np
import pytest

from paper_2601_08217_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def _setup(B, N, n_ue, pool):
    cells = [dict(sample_rate_hz=61.44e6, n_ant=2, max_samples=N, ul_sigma=0.05, ul_noise_off=[3, 77, 0, 0])]
    ch = B.Channel(cells, n_ue, 64 << 20, "ci16", pool)
    ch.set_tuning(ul_group=2)  # several groups, so the partials are used
    ids = []
    for u in range(n_ue):
        uid = ch.add_ue(cell=0, n_taps=12, n_tx=1, n_rx=1, mode="linear", snapshot_period=64)
        snaps = W.rayleigh_snapshots(31, W.link_key(u, "ul"), 130, 2, 1, W.exp_pdp(12, total=1.0 / n_ue), "f32")
        ch.set_taps(uid, "ul", 0, snaps)
        ids.append(uid)
    return ch, ids


def test_noalloc_ul_matches_apply_ul_over_two_calls():
    import torch
    from paper_2601_08217_amd import binding as B
    N, n_ue = 5000, 5
    pool = W.noise_pool(31, 1 << 16)
    a, ids_a = _setup(B, N, n_ue, pool)
    b, ids_b = _setup(B, N, n_ue, pool)
    assert ids_a == ids_b
    x = [torch.from_numpy(W.iq_block(31, u, 0, 1, N, "ci16")).to("cuda:0") for u in range(n_ue)]
    calls = [(N, n_ue), (3001, 3)]
    outs = []
    torch.cuda.synchronize()
    free0 = None
    for n_samples, k in calls:
        za = torch.zeros((2, n_samples, 2), dtype=torch.int16, device="cuda:0")
        zb = torch.zeros_like(za)
        a.apply_ul(0, n_samples, ids_a[:k], [t.data_ptr() for t in x[:k]], za.data_ptr())
        a.sync()
        if free0 is None:
            free0 = torch.cuda.mem_get_info()[0]
        b.apply_ul_noalloc(0, n_samples, ids_b[:k], [t.data_ptr() for t in x[:k]], zb.data_ptr())
        b.sync()
        outs.append((za.cpu().numpy(), zb.cpu().numpy()))
    free1 = torch.cuda.mem_get_info()[0]
    for i, (za, zb) in enumerate(outs):
        assert np.abs(za.astype(np.int32)).max() > 0, i
        assert np.array_equal(za, zb), i
    assert free1 == free0, (free0, free1)
    a.close()
    b.close()


def test_noalloc_ul_refuses_partials_beyond_the_scratch():
    """8 groups x 4 antennas x 65,536 samples x 8 B is exactly the 16 MiB
    scratch and runs; a ninth group is refused before any work."""
    import torch
    from paper_2601_08217_amd import binding as B
    N, n_ue = 65536, 9
    pool = W.noise_pool(32, 1 << 16)
    cells = [dict(sample_rate_hz=122.88e6, n_ant=4, max_samples=N)]
    ch = B.Channel(cells, n_ue, 512 << 20, "cf32", pool)
    ch.set_tuning(ul_group=1)
    ids = [ch.add_ue(cell=0, n_taps=1, n_tx=1, mode="hold", snapshot_period=1 << 20) for _ in range(n_ue)]
    for u in ids:
        ch.set_taps(u, "ul", 0, np.ones((2, 4, 1, 1), np.complex64))
    x = torch.ones((1, N), dtype=torch.complex64, device="cuda:0")
    z = torch.zeros((4, N), dtype=torch.complex64, device="cuda:0")
    ch.apply_ul_noalloc(0, N, ids[:8], [x.data_ptr()] * 8, z.data_ptr())
    ch.sync()
    assert np.allclose(z.cpu().numpy(), 8.0), "eight unit taps on a unit input"
    with pytest.raises(B.TTError):
        ch.apply_ul_noalloc(0, N, ids, [x.data_ptr()] * n_ue, z.data_ptr())
    ch.close()
