"""The streaming pipeline (snapshots in pinned host memory, copied in, estimated and copied out on
several slots with their own streams) against nssdoa_estimate on device-resident data: the same
peaks, counts, status and spectrum, bit for bit, for a run of submissions with different snapshots
and every slot reused; waits in and out of order; argument errors; the batch outlives it.
"""

import numpy as np
import pytest

from synth import make_frames
from gpu_common import frameset_inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _sets(n_sets, prec):
    # frame sets of one layout (same M, N, D, grid per frame position), different snapshots
    out = []
    for k in range(n_sets):
        fs = make_frames("c2", n_frames=8, N=1024, grid_step=0.05, start=900 + 8 * k)
        out.append(fs)
    return out


@pytest.mark.parametrize("depth,prec,with_spec", [(2, "c64", True), (3, "c64", False), (2, "c128", True)])
def test_pipeline_equals_resident_estimate(depth, prec, with_spec):
    _need_gpu()
    import paper_2007_14135_amd as nd
    from paper_2007_14135_amd.runner import prepare
    print("pipeline: depth %d %s spectrum %s" % (depth, prec, with_spec), flush=True)
    sets = _sets(5, prec)
    if prec == "c128":
        from synth.frames import pack_frames
        sets = [pack_frames(fs.frames, dtype=np.complex128) for fs in sets]
    arrays, grids, frames, X0 = frameset_inputs(sets[0])
    db = prepare(arrays, grids, frames, X0, "music", prec, 4, with_spectrum=True)
    pipe = nd.Pipeline(db.batch, depth)
    F, mD = len(sets[0]), 4
    ftype = np.float64 if prec == "c128" else np.float32
    hosts = []
    tickets = []
    for fs in sets:
        Xh = torch.from_numpy(np.ascontiguousarray(fs.X_flat).view(ftype).copy()).pin_memory()
        pk = torch.empty(F * mD * 32, dtype=torch.uint8).pin_memory()
        npk = torch.empty(F, dtype=torch.int32).pin_memory()
        st = torch.empty(F, dtype=torch.int32).pin_memory()
        sp = torch.empty(db.spectrum.numel(), dtype=db.spectrum.dtype).pin_memory() if with_spec else None
        hosts.append((Xh, pk, npk, st, sp))
        tickets.append(pipe.submit(Xh, pk, npk, st, sp))
    assert tickets == list(range(len(sets)))
    for t in reversed(tickets):                 # waits in any order
        pipe.wait(t)
    for fs, (Xh, pk, npk, st, sp) in zip(sets, hosts):
        db.X.copy_(Xh.to(db.X.device))
        db.run()
        ref = db.host_results()
        torch.cuda.synchronize()
        assert np.array_equal(npk.numpy(), ref["npeaks"])
        assert np.array_equal(st.numpy().astype(np.uint32), ref["status"])
        assert pk.numpy().tobytes() == db.peaks.cpu().numpy().tobytes()
        if with_spec:
            assert np.array_equal(sp.numpy(), db.spectrum.cpu().numpy(), equal_nan=True)
    pipe.close()


def test_pipeline_arguments_and_lifetime():
    _need_gpu()
    import paper_2007_14135_amd as nd
    from paper_2007_14135_amd import _abi
    from paper_2007_14135_amd.runner import prepare
    fs = make_frames("c2", n_frames=2, N=256, grid_step=0.1, start=990)
    arrays, grids, frames, X0 = frameset_inputs(fs)
    db = prepare(arrays, grids, frames, X0, "music", "c64", 4)
    for bad in (0, 9):
        with pytest.raises(_abi.NssdoaError) as e:
            nd.Pipeline(db.batch, bad)
        assert e.value.status == _abi.EINVAL
    pipe = nd.Pipeline(db.batch, 2)
    with pytest.raises(_abi.NssdoaError) as e:
        pipe.wait(0)                            # never issued
    assert e.value.status == _abi.EINVAL
    with pytest.raises(_abi.NssdoaError) as e:
        db.batch.close()                        # the pipeline still uses the batch
    assert e.value.status == _abi.ESTATE
    pipe.close()
    db.batch.close()
