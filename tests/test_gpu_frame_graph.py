"""A whole KK frame (kk_decompose + kk_beamform with the Eq. 9 intensity) captured as one HIP
graph: every replay, with unrelated eager work between replays, gives the eager frame's images
bit for bit, and the replayed images match the FP64 oracle at sampled pixels."""
import numpy as np
import pytest

from paper_2603_22496_amd import configs as C
from tests import oracle_ref as OR

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kk():
    import torch
    from paper_2603_22496_amd import kk as K
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    K.lib()
    return K


def _frame_buffers(K, w, ds, torch):
    su = K.make_setup(w)
    S = su.sel["S"]
    dev = torch.device("cuda", 0)
    b = dict(su=su, rf=K.to_device(ds.rf), shift=K.to_device(su.luts["shift"]), plan=K.to_device(su.plan),
             rt=torch.empty((w.N, su.M, w.T), dtype=torch.complex64, device=dev),
             ws=torch.empty(K.decompose_workspace_bytes(su.geom, w.N, su.M, su.tpad), dtype=torch.uint8, device=dev),
             img=torch.empty((S, w.X, w.Z), dtype=torch.complex64, device=dev),
             inten=torch.empty((w.X, w.Z), dtype=torch.float32, device=dev),
             bws=torch.empty(max(1, K.beamform_workspace_bytes(su.plan)), dtype=torch.uint8, device=dev))
    return b


def _frame(K, b):
    su = b["su"]
    K.decompose(b["rf"], su.geom, b["shift"], su.M, su.tpad, out=b["rt"], ws=b["ws"])
    K.beamform(b["rt"], su.plan, b["plan"], image=b["img"], intensity=b["inten"], mode=K.COMPOUND_INCOHERENT,
               ws=b["bws"])


@pytest.mark.parametrize("case", ["tiny", "vernier"])
def test_frame_graph_replays_equal_eager(kk, case):
    import torch
    if case == "tiny":
        w, ds = C.TINY, C.tiny_dataset(3)
        w2, ds2 = C.TINY, C.tiny_dataset(4)
    else:
        w, ds = C.VERNIER, C.speckle_dataset(C.VERNIER, seed=5, n_scat=3000)
        w2, ds2 = C.TINY, C.tiny_dataset(5)
    print("frame graph case", case, flush=True)
    b = _frame_buffers(kk, w, ds, torch)
    other = _frame_buffers(kk, w2, ds2, torch)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        _frame(kk, b)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    ref_img, ref_int = b["img"].cpu().numpy(), b["inten"].cpu().numpy()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        _frame(kk, b)
    for rep in range(3):
        b["img"].zero_()
        b["inten"].zero_()
        b["rt"].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(b["img"].cpu().numpy(), ref_img, err_msg="replay %d" % rep)
        np.testing.assert_array_equal(b["inten"].cpu().numpy(), ref_int, err_msg="replay %d" % rep)
        _frame(kk, other)                          # unrelated eager work between replays
        torch.cuda.synchronize()
    del g
    # the replayed frame against the FP64 oracle at sampled pixels
    su = b["su"]
    rng = np.random.default_rng(0)
    xi, zi = rng.integers(0, w.X, 200), rng.integers(0, w.Z, 200)
    ref = OR.tables(su, w).kk_image(ds.rf, pixels=(xi, zi))
    got = ref_img[:, xi, zi]
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-5


def test_frames_in_flight_on_separate_streams(kk):
    """Three different frames enqueued on three streams at once (each with its own buffers) give
    the images each gives alone: the library keeps no state between calls."""
    import torch
    print("frames in flight on three streams", flush=True)
    cases = [(C.VERNIER, C.speckle_dataset(C.VERNIER, seed=11 + k, n_scat=2000)) for k in range(3)]
    bufs = [_frame_buffers(kk, w, ds, torch) for w, ds in cases]
    alone = []
    for b in bufs:
        _frame(kk, b)
        torch.cuda.synchronize()
        alone.append((b["img"].cpu().numpy(), b["inten"].cpu().numpy()))
        b["img"].zero_()
        b["inten"].zero_()
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in bufs]
    for rep in range(3):
        for b, st in zip(bufs, streams):
            su = b["su"]
            kk.decompose(b["rf"], su.geom, b["shift"], su.M, su.tpad, out=b["rt"], ws=b["ws"], stream=st)
            kk.beamform(b["rt"], su.plan, b["plan"], image=b["img"], intensity=b["inten"],
                        mode=kk.COMPOUND_INCOHERENT, ws=b["bws"], stream=st)
        torch.cuda.synchronize()
        for k, b in enumerate(bufs):
            np.testing.assert_array_equal(b["img"].cpu().numpy(), alone[k][0], err_msg="frame %d rep %d" % (k, rep))
            np.testing.assert_array_equal(b["inten"].cpu().numpy(), alone[k][1], err_msg="frame %d rep %d" % (k, rep))
            b["img"].zero_()
            b["inten"].zero_()
        torch.cuda.synchronize()
