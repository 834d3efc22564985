"""ss_sort_frame_noalloc (workspace in the library's own device array) on
the GPU, through the C ABI: two calls in a row, the second on a smaller
frame, each equal bit for bit to ss_sort_frame with a caller workspace."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2511_16298_amd as ss  # noqa: E402
from paper_2511_16298_amd import _abi  # noqa: E402


def outputs(w, h, n, capacity, dev):
    tx, ty, _ = ss.geometry(w, h)
    o = {"keys": torch.empty(max(capacity, 1), dtype=torch.int64, device=dev),
         "values": torch.empty(max(capacity, 1), dtype=torch.int32, device=dev),
         "ranges": torch.empty((tx * ty, 2), dtype=torch.int32, device=dev),
         "num_pairs": torch.zeros(1, dtype=torch.int32, device=dev),
         "status": torch.zeros(1, dtype=torch.int32, device=dev)}
    c = _abi.ss_frame_out()
    c.pair_capacity = capacity
    c.keys, c.values = o["keys"].data_ptr(), o["values"].data_ptr()
    c.tile_ranges = o["ranges"].data_ptr()
    c.num_pairs, c.status = o["num_pairs"].data_ptr(), o["status"].data_ptr()
    return o, c


# the second case keeps both calls on the multi-kernel path (a full-HD
# frame of 3x10^5 Gaussians after one of 10^6), so the smaller call runs in
# the array the larger one left behind
WORKLOADS = dict(synth.FRAME_WORKLOADS)
WORKLOADS["fullhd-300k"] = (synth.scaled(synth.FRAME_WORKLOADS["fullhd-1m"][0], 300_000),
                            synth.FRAME_WORKLOADS["fullhd-1m"][1] + 17)


@pytest.mark.parametrize("order", [("fullhd-1m", "small-256x256"), ("fullhd-1m", "fullhd-300k")])
def test_noalloc_equals_sort_frame_twice(order):
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream()
    for name in order:
        spec, seed = WORKLOADS[name]
        rec = synth.make_frame(spec, seed)
        d = ss.records_to_device(rec, dev)
        _, _, m_t, s_t = ss.count_pairs(d, spec.width, spec.height)
        assert int(s_t.item()) == 0
        cap = int(m_t.item()) & 0xFFFFFFFF
        print(f"noalloc: {name} N={len(rec)} M={cap}", flush=True)
        ref = ss.FrameSorter(spec.width, spec.height, len(rec), cap, device=dev)
        ref(d, stream)
        o, c = outputs(spec.width, spec.height, len(rec), cap, dev)
        f = ss._frame(d, spec.width, spec.height)
        st = _abi.ss_sort_frame_noalloc(f, c, stream.cuda_stream)
        assert st == _abi.SS_OK, _abi.status_string(st)
        torch.cuda.synchronize()
        assert int(o["status"].item()) == 0 and (int(o["num_pairs"].item()) & 0xFFFFFFFF) == cap
        r_st, r_m = ref.out.result()
        assert r_st == 0 and r_m == cap
        assert torch.equal(o["keys"][:cap], ref.out.keys[:cap])
        assert torch.equal(o["values"][:cap], ref.out.values[:cap])
        assert torch.equal(o["ranges"], ref.out.tile_ranges)
