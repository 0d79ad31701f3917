"""The grouped (graph-captured) step of the batched engine."""
import os

import numpy as np
import pytest
import torch

import paper_2104_14101_amd as aes
import synth
from oracle import reference

from _helpers import to_dev

pytestmark = pytest.mark.gpu


def _probs(specs, nrhs, seed0):
    out = []
    for i, (n, d, nu) in enumerate(specs):
        P = synth.make_problem(n, d, "geo:0.98", nu, nrhs=nrhs, seed=seed0 + i)
        out.append(dict(A=to_dev(P["A"]), b=to_dev(P["b"]), nu=nu, A_np=P["A"], b_np=P["b"], V=P["V"],
                        sigma=P["sigma"]))
    return out


@pytest.mark.parametrize("precision,method", [("mixed_fp32", "pcg"), ("fp64", "pcg"), ("fp64", "ihs"),
                                              ("mixed", "polyak")])
def test_graph_replays_equal_eager_steps(precision, method):
    # the captured step replayed once per step (with eager resizes and refinement between the
    # replays) gives bit-identical results to the same launches enqueued eagerly every step
    specs = [(4096, 256, 1e-1), (3000, 520, 1e-3), (2048, 1024, 1e-2), (5000, 1300, 3e-3)]
    probs = _probs(specs, 8, 70)
    kw = dict(tol=1e-10, precision=precision, method=method, m_init=16, seed=9)
    if method == "polyak":
        kw.update(max_iter=400)
    res_g = aes.solve_batched(probs, **kw)
    os.environ["AES_BATCH_GRAPH"] = "0"
    try:
        res_e = aes.solve_batched(probs, **kw)
    finally:
        del os.environ["AES_BATCH_GRAPH"]
    for p, ((xg, ig), (xe, ie)) in enumerate(zip(res_g, res_e)):
        assert ig["status"] == "ok" and ie["status"] == "ok", (p, ig, ie)
        assert ig["iterations"] == ie["iterations"] and ig["final_m"] == ie["final_m"]
        assert torch.equal(xg, xe), p
        xr = reference.reference_solution(probs[p]["A_np"], probs[p]["b_np"], probs[p]["nu"],
                                          spectral=(probs[p]["V"], probs[p]["sigma"]))
        assert np.all(reference.rel_error(xg.cpu().numpy(), xr) <= 1e-10), p


def test_tuner_times_plans_and_rejects_inapplicable_ones():
    import ctypes

    from paper_2104_14101_amd import _binding as B

    lib = B.load()
    dev = torch.device("cuda:0")
    h = aes._handle(dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    A = torch.randn((4096, 512), dtype=torch.float64, device=dev)

    def t(prec, twopass, rows, d=512, a=A):
        ms = ctypes.c_double(-1.0)
        st = lib.aes_tune_hp(h, stream, a.shape[0], d, 32, ctypes.c_void_p(a.data_ptr()), a.shape[1],
                             B.PRECISIONS[prec], twopass, rows, 3, ctypes.byref(ms))
        return st, ms.value

    for prec in ("fp64", "mixed_fp32"):
        for twopass in (0, 1):
            st, ms = t(prec, twopass, 256)
            assert st == B.AES_OK and ms > 0.0
    wide = torch.randn((512, 1536), dtype=torch.float64, device=dev)
    assert t("fp64", 0, 256, 1536, wide)[0] == B.AES_ERR_INVALID_ARG   # fused FP64 takes d <= 1024
    assert t("fp64", 1, 256, 1536, wide)[0] == B.AES_OK
    assert t("fp64", 0, 24)[0] == B.AES_ERR_INVALID_ARG                # rows not a multiple of 16
