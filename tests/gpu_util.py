"""Helpers of the GPU tests: run the HIP build and compare with the oracle."""
import numpy as np

import oracle


def gpu_labels(row, col, w, order, **kw):
    from paper_1907_00140_amd import chl
    L = chl.build(row, col, w, order, **kw)
    off, hub, dist = L.export("cpu")
    return L, off.numpy(), hub.numpy(), dist.numpy()


def assert_same_labels(off, hub, dist, ref, where=""):
    """Bit-exact comparison with an oracle Labels object."""
    assert np.array_equal(off, ref.offsets), where + ": offsets differ"
    assert np.array_equal(hub, ref.hub_pos), where + ": hubs differ"
    assert np.array_equal(dist.astype(np.int64), ref.dist), where + ": distances differ"


def per_root_from_export(off, hub, dist, order, roots):
    """Labels of the given roots (rank positions) from an exported labeling:
    {root: (vertices sorted, distances)}."""
    n = len(off) - 1
    v_of = np.repeat(np.arange(n, dtype=np.int32), np.diff(off))
    out = {}
    sel = np.isin(hub, np.asarray(roots, dtype=np.int32))
    hv, vv, dv = hub[sel], v_of[sel], dist[sel].astype(np.int64)
    for r in roots:
        m = hv == r
        idx = np.argsort(vv[m], kind="stable")
        out[int(r)] = (vv[m][idx], dv[m][idx])
    return out
