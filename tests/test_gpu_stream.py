"""Streaming labels in z-slabs (fof_stream_counts / fof_stream_workspace_bytes /
fof_link_stream, paper Sec. 2.3: slabs with ghost layers, components fused through the
particles they share): the labels must equal the oracle's and the in-core fof_link's bit
for bit, for any number of slabs, including clumps that straddle a slab face and the
periodic z boundary; the workspace holds one slab at a time."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import run_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def stream_labels(pos, L, b, nslab, tune=None):
    import torch
    from paper_2510_26851_amd import Stream

    t = torch.from_numpy(np.ascontiguousarray(pos)).cuda()
    st = Stream(t, L, b, nslab=nslab, tune=tune)
    root = st.labels()
    torch.cuda.synchronize()
    assert int(st.counts.sum()) >= pos.shape[0]
    return root.cpu().numpy()[:pos.shape[0]], st.status(), st


def straddling_box(seed=7):
    """Uniform particles plus Gaussian clumps centred on slab faces (z = k L / 8) and on the
    periodic boundary z = 0, in L = 24 (b from the mean spacing)."""
    rng = np.random.default_rng(seed)
    L = 24.0
    parts = [rng.random((20000, 3)) * L]
    for k in range(8):
        c = np.array([rng.random() * L, rng.random() * L, k * L / 8])
        parts.append(c + 0.25 * rng.standard_normal((1500, 3)))
    pos = W.wrap_to_f32(np.concatenate(parts), (L, L, L))
    return pos, L, W.linking_length(0.2, L, pos.shape[0])


@pytest.mark.parametrize("nslab", [1, 2, 3, 8, 13])
def test_stream_config0(nslab):
    box = W.config0()
    say(f"stream config0 nslab={nslab}")
    ref, _ = oracle.fof(box.pos, box.L, box.b)
    got, status, _ = stream_labels(box.pos, box.L, box.b, nslab)
    assert status == 0
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("nslab,tune", [(8, None), (4, dict(dense_threshold=8)),
                                        (6, dict(dense_threshold=-1))])
def test_stream_clumps_on_slab_faces(nslab, tune):
    pos, L, b = straddling_box()
    say(f"stream straddling clumps nslab={nslab} tune={tune}")
    ref, _ = oracle.fof(pos, L, b)
    got, status, _ = stream_labels(pos, L, b, nslab, tune=tune)
    assert status == 0
    np.testing.assert_array_equal(got, ref)
    in_core, _, _ = run_gpu(pos, L, b, 2)
    np.testing.assert_array_equal(got, in_core)


def test_stream_status_bits():
    import torch
    from paper_2510_26851_amd import Stream

    box = W.config0()
    pos = box.pos.copy()
    pos[5, 0] = np.float32(box.L[0])                # x == L: out of range
    st = Stream(torch.from_numpy(pos).cuda(), box.L, box.b, nslab=4)
    st.labels()
    torch.cuda.synchronize()
    assert st.status() & 1
    say("stream with a count that is not the slab's")
    st = Stream(torch.from_numpy(box.pos).cuda(), box.L, box.b, nslab=4)
    st.counts[2] -= 1                               # smaller than the slab: flagged
    st.labels()
    torch.cuda.synchronize()
    assert st.status() & 16


def test_stream_rejects_bad_slabs():
    import torch
    from paper_2510_26851_amd import Stream, _lib

    box = W.config0()
    t = torch.from_numpy(box.pos).cuda()
    with pytest.raises(_lib.FoFError):
        Stream(t, box.L, box.b, nslab=60)            # slabs thinner than 3 b
    with pytest.raises(_lib.FoFError):
        Stream(t, box.L, box.b, nslab=0)
