"""The no-allocation entry point captured in a HIP graph, the use it exists
for: a caller under stream capture cannot allocate.  The captured loop
hafnian is replayed several times with eager work of the program (fills of
the outputs, another loop hafnian) between the replays, and every replay must
equal the eager call bit for bit: the same kernels run in the same order on
the same inputs."""
import numpy as np
import pytest

import paper_2010_15595_amd as gbs
from paper_2010_15595_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [gbs.GBS_FP64, gbs.GBS_FP32_COMP])
def test_noalloc_replays_under_graph_capture(prec):
    import torch

    gbs.init(0)
    dev = torch.device("cuda:0")
    st = workloads.config3(30)
    At = torch.from_numpy(gbs.expand(st["B"], st["gamma"], st["pattern"])).to(dev)
    other = torch.from_numpy(workloads.random_normal_symmetric(24, seed=77, scale=0.5)).to(dev)
    ref = torch.zeros(1, dtype=torch.complex128, device=dev)
    ref_ab = torch.zeros(1, dtype=torch.float64, device=dev)
    gbs.lhaf_device_noalloc(At, ref, ref_ab, prec=prec)
    torch.cuda.synchronize()
    ref_v, ref_a = complex(ref.cpu()[0]), float(ref_ab.cpu()[0])

    out = torch.zeros(1, dtype=torch.complex128, device=dev)
    ab = torch.zeros(1, dtype=torch.float64, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up off the default stream, as for any captured work
        gbs.lhaf_device_noalloc(At, out, ab, prec=prec)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gbs.lhaf_device_noalloc(At, out, ab, prec=prec)
    scratch_out = torch.zeros(1, dtype=torch.complex128, device=dev)
    for k in range(4):
        out.fill_(complex(np.nan, np.nan))
        ab.fill_(np.nan)
        gbs.lhaf_device_noalloc(other, scratch_out, prec=prec)  # eager use of the same scratch array
        g.replay()
        torch.cuda.synchronize()
        got_v, got_a = complex(out.cpu()[0]), float(ab.cpu()[0])
        print(f"[noalloc graph prec={prec}] replay {k}: {got_v!r} vs eager {ref_v!r}", flush=True)
        assert got_v == ref_v and got_a == ref_a
