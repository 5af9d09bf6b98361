"""The metrics entry point that allocates nothing (its scratch is a buffer
built into the library) gives exactly what erbf_surface_metrics gives with a
caller's scratch, on two calls in a row, the second smaller than the first;
sizes past its limit are refused."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _sets(rng, nt, nr):
    def one(n):
        p = rng.normal(size=(n, 3))
        p /= np.linalg.norm(p, axis=1, keepdims=True)
        nrm = p + 0.05 * rng.normal(size=(n, 3))
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        return (0.5 * p).astype(np.float32), nrm.astype(np.float32)
    return one(nt) + one(nr)


def test_noalloc_metrics_equal_the_scratch_argument_call():
    import torch
    from paper_2505_02350_amd import _lib as L
    from paper_2505_02350_amd import core
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(91)
    for nt, nr in ((40000, 30011), (777, 1234)):
        print(f"metrics no-alloc vs scratch argument, nt={nt} nr={nr}", flush=True)
        Pt, Nt, Pr, Nr = (torch.from_numpy(x).to(dev) for x in _sets(rng, nt, nr))
        ref = core.erbf_surface_metrics(Pt, Nt, Pr, Nr)
        got = core.erbf_surface_metrics_noalloc(Pt, Nt, Pr, Nr)
        assert got == ref, (got, ref)
    lib = L.load()
    big = 1 << 20
    rc = lib.erbf_surface_metrics_noalloc(Pt.data_ptr(), Nt.data_ptr(), big - 10, Pr.data_ptr(), Nr.data_ptr(), 11,
                                          Pt.data_ptr(), None)
    assert rc == L.ERBF_ERR_INVALID_ARG and b"scratch limit" in lib.erbf_last_error()
