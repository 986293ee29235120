"""Parity at the benchmark's full size: n = 100,000 amplicon reads of 200
references, k = 100, oversample 20, q = 2, in the launch configuration that
bench.py times.  The reference is the FP64 oracle run block-row-wise on the
host (same method, same test matrix), so this is element-by-element parity on
the eigenvalues and coordinates, plus the centring statistics of every row and
column and the Rayleigh quotients of the returned axes against the exact G.
Needs about 45 GB of host memory and a couple of minutes of host compute.
"""
import time

import numpy as np
import pytest

from gpu_util import procrustes_err, rel_eig_err, say

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1803_02272_amd as mds  # noqa: E402
from paper_1803_02272_amd import _capi  # noqa: E402
from oracle import mds_oracle_large as OL  # noqa: E402
from workloads import gpu as WG  # noqa: E402

N, REFS, K, P, Q, SEED = 100000, 200, 100, 20, 2, 0


@pytest.mark.timeout(1000)
def test_paper_scale_parity():
    t0 = time.time()
    say(f"[fullsize] generating amplicon D n={N} refs={REFS} on the GPU")
    D = WG.amplicon_distances(N, REFS, seed=SEED)
    res = {}
    for form in ("bf16", "fp32"):
        say(f"[fullsize] GPU run form={form}")
        plan = mds.Plan(N, K, P, Q, SEED, form=form)
        coords, eig = plan.run(D)
        info = plan.info()
        assert info["status"] == 0, info
        res[form] = {
            "X": coords.cpu().numpy(), "eig": eig.cpu().numpy(), "info": info,
            "r": plan.buffer(_capi.BUF_ROWMEAN).double().cpu().numpy()[:, 0].copy(),
            "c": plan.buffer(_capi.BUF_COLMEAN).double().cpu().numpy()[:, 0].copy(),
        }
        plan.close()
        torch.cuda.empty_cache()
    say(f"[fullsize] copying D to the host ({time.time() - t0:.0f} s)")
    Dh = D.cpu().numpy()
    del D
    torch.cuda.empty_cache()
    ref = OL.rand_mds_blocked(Dh, K, P, Q, SEED, form="fp64",
                              progress=lambda m: say(f"[fullsize] oracle: {m} ({time.time() - t0:.0f} s)"))
    r, c, m = ref["stats"]
    for form, rr in res.items():
        assert np.max(np.abs(rr["r"] - r) / r) < 1e-13
        assert np.max(np.abs(rr["c"] - c) / c) < 1e-13
    e_bf = rel_eig_err(res["bf16"]["eig"], ref["eigvals"])
    e_32 = rel_eig_err(res["fp32"]["eig"], ref["eigvals"])
    c_bf = procrustes_err(res["bf16"]["X"], ref["coords"])
    c_32 = procrustes_err(res["fp32"]["X"], ref["coords"])
    say(f"[fullsize] eig rel err bf16 {e_bf:.3e} fp32 {e_32:.3e}; coords procrustes bf16 {c_bf:.3e} fp32 {c_32:.3e}")
    assert e_bf < 1e-3
    assert e_32 < 1e-5
    assert c_bf < 5e-3
    assert c_32 < 1e-3
    # Rayleigh quotients of the bf16 form's axes against the exact G
    X = res["bf16"]["X"]
    th = res["bf16"]["eig"]
    U = X / np.sqrt(th)[None, :]
    assert np.max(np.abs(U.T @ U - np.eye(K))) < 1e-10
    GU = OL.gram_apply_blocked(Dh, ref["stats"], U)
    rq = np.einsum("ia,ia->a", U, GU)
    say(f"[fullsize] Rayleigh quotient rel err {np.max(np.abs(rq - th) / th):.3e} ({time.time() - t0:.0f} s)")
    assert np.max(np.abs(rq - th) / th) < 1e-5
