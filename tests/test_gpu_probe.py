"""The random-gather probe reads exactly the records it claims (the index
sequence and the sums are reproduced on the host), so the ceiling it
measures is the one documented for it."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def host_probe(table, rec16, in_flight, n_waves, iters, seed):
    n_rec = table.shape[0] // rec16
    out = np.zeros(n_waves * 64, np.float32)
    for lane in range(n_waves * 64):
        M64 = (1 << 64) - 1
        s = (((lane + 1) * 0x9E3779B97F4A7C15) & M64) ^ (seed << 17)
        if s == 0:
            s = 0x6D2B79F5
        acc = np.float32(0)
        for _ in range(iters):
            recs = []
            for _u in range(in_flight):
                s ^= (s << 13) & M64
                s ^= s >> 7
                s ^= (s << 17) & M64
                r = (s * n_rec) >> 64
                recs.append(table[r * rec16:(r + 1) * rec16])
            for v in recs:
                for x, y, z, w in v:
                    acc = np.float32(acc + np.float32(np.float32(x + y) + np.float32(z + w)))
        out[lane] = acc
    return out


@pytest.mark.parametrize("rec,in_flight", [(16, 1), (64, 4), (128, 2)])
def test_gather_probe_reads_the_drawn_records(rec, in_flight):
    import torch
    from paper_2111_08744_amd import _abi
    L = _abi.lib()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(7)
    n_rec = 997                                    # not a power of two
    table = rng.standard_normal((n_rec * rec // 16, 4)).astype(np.float32)
    t = torch.from_numpy(table).to(dev)
    n_waves, iters, seed = 3, 5, 0xABCDEF
    out = torch.full((n_waves * 64,), float("nan"), dtype=torch.float32, device=dev)
    print(f"gather probe: {rec} B records, {in_flight} in flight", flush=True)
    rc = L.mpath_gather_probe(t.data_ptr(), t.numel() * 4, rec, in_flight, n_waves, iters, seed,
                              out.data_ptr(), torch.cuda.current_stream(dev).cuda_stream)
    _abi.check(rc, "mpath_gather_probe")
    got = out.cpu().numpy()
    want = host_probe(table, rec // 16, in_flight, n_waves, iters, seed)
    np.testing.assert_array_equal(got, want)
