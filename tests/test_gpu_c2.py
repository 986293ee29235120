"""Parity on the plain FP32 amplicon workload: 50 random ACGT references of
length 400, n = 20,000 reads (each a uniformly chosen reference with i.i.d.
substitutions at a per-read rate uniform in 1-5%), D = Hamming / 400 in fp32,
k = 50, oversample 10, q = 2.  The reference is the FP64 oracle (same method,
same test matrix) on the same D, and the oracle run with each form's operand
roundings.  The fp32 form is this workload's form; the bf16 form and the fp32
form with split passes are checked as well, the bf16 form against the plain
oracle at its 1e-3 bar.
"""
import numpy as np
import pytest

from gpu_util import procrustes_err, rel_eig_err, say

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
import paper_1803_02272_amd as mds  # noqa: E402
import workloads as W  # noqa: E402

N, REFS, K, P, Q, SEED = 20000, 50, 50, 10, 2, 0


@pytest.mark.timeout(900)
def test_c2_amplicon_n20000():
    reads, _ = W.amplicon_reads(N, REFS, seed=SEED)
    D = W.hamming_distances(reads)  # fp32, exact counts / 400
    assert D.dtype == np.float32 and D.shape == (N, N)
    say(f"[c2] oracle n={N} k={K} p={P} q={Q}")
    ref = O.rand_mds(D, K, P, Q, SEED)
    ref32 = O.rand_mds(D, K, P, Q, SEED, form="fp32")
    ref16 = O.rand_mds(D, K, P, Q, SEED, form="bf16")
    Dg = torch.from_numpy(D).cuda()
    for form, split, matched, bar_matched in (("fp32", False, ref32, 1e-5), ("fp32", True, ref32, 1e-5),
                                              ("bf16", False, ref16, 1e-4)):
        plan = mds.Plan(N, K, P, Q, SEED, form=form, split_fp32=split)
        coords, eig = plan.run(Dg)
        info = plan.info()
        assert info["status"] == 0, info
        eig, X = eig.cpu().numpy(), coords.cpu().numpy()
        err, merr = rel_eig_err(eig, ref["eigvals"]), rel_eig_err(eig, matched["eigvals"])
        cerr = procrustes_err(X, ref["coords"])
        say(f"[c2] form={form}{' split' if split else ''}: eig rel err vs fp64 {err:.3e}, vs matched {merr:.3e},"
            f" coords procrustes {cerr:.3e}")
        assert merr < bar_matched
        if form == "fp32":
            assert err < 1e-5
            assert cerr < 1e-3
        else:  # bf16 form (fp32 end passes) against the plain fp64 oracle
            assert err < 1e-3
            assert cerr < 5e-3
        plan.close()
