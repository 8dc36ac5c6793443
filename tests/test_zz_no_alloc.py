"""hme_compute_noalloc (the entry point that allocates nothing) against hme_compute, through
the C ABI: bitwise the same |M|^2 on two calls in a row, the second with a smaller batch, for
the process whose kernels use the workspace (gg -> ttbar ggg in single and double precision,
sub-batches of the 256 MiB scratch) and for one that uses none (gg -> ttbar gg)."""
import numpy as np
import pytest

import paper_2507_21039_amd as hme
from workloads import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

AS = 0.118


def _both(h, p):
    t = torch.from_numpy(np.ascontiguousarray(p)).cuda()
    n = p.shape[0]
    ref = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    got = torch.full((n,), -2.0, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    h.compute_ptr(AS, n, t.data_ptr(), ref.data_ptr(), s)
    h.compute_noalloc_ptr(AS, n, t.data_ptr(), got.data_ptr(), s)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


@pytest.mark.parametrize("key,proc,prec,sizes", [
    ("ggttggg", hme.GGTTGGG, hme.MIXED_FAST, (1000, 333)),
    # double workspace: 160-event sub-batches of the scratch array, FP64 colour sum by fold
    ("ggttggg", hme.GGTTGGG, hme.FP64, (400, 97)),
    ("ggttgg", hme.GGTTGG, hme.FP64, (3001, 129)),
])
def test_noalloc_equals_compute(card, key, proc, prec, sizes):
    print(f"[gpu] noalloc {key} sizes {sizes}", flush=True)
    with hme.Handle(proc, card, prec) as h:
        for k, n in enumerate(sizes):
            p = configs.WORKLOADS[key].momenta(n, first_event=7 * k)
            ref, got = _both(h, p)
            assert np.all(np.isfinite(ref)) and np.all(ref > 0)
            assert np.array_equal(got, ref), (key, n)


def test_noalloc_arguments(card):
    with hme.Handle(hme.GGTT, card, hme.FP64) as h:
        t = torch.zeros((8, 4, 4), dtype=torch.float64, device="cuda")
        out = torch.zeros(8, dtype=torch.float64, device="cuda")
        s = torch.cuda.current_stream().cuda_stream
        h.compute_noalloc_ptr(AS, 0, t.data_ptr(), out.data_ptr(), s)  # no-op
        with pytest.raises(hme.HmeError) as e:
            h.compute_noalloc_ptr(AS, -1, t.data_ptr(), out.data_ptr(), s)
        assert e.value.code == hme.HME_E_ARG
        with pytest.raises(hme.HmeError):
            h.compute_noalloc_ptr(AS, 8, t.data_ptr() + 4, out.data_ptr(), s)
