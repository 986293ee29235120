"""GPU parity: every stage of the HIP path against the FP64 CPU oracle on the
same seeded inputs, through the C ABI.

Sizes span several tiles of every kernel plus ragged tails (n not a multiple
of 4, 256 or 1024; odd l; l above the LDS limit of the small kernels).
Bars: fp64 form 1e-10 relative on eigenvalues, fp32 form 1e-5, bf16 form
1e-3; coordinates after sign + orthogonal Procrustes alignment.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import bf16_round, procrustes_err, rel_eig_err, say, sign_aligned_err, span_cos_min

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - collected on CPU only
    pytest.skip("no GPU", allow_module_level=True)

import paper_1803_02272_amd as mds  # noqa: E402
from paper_1803_02272_amd import _capi  # noqa: E402

# bars against the plain fp64 oracle (the stated targets): relative error
# per eigenvalue over the top k, coordinates after sign + Procrustes.  The
# bf16 form's first and last range passes are fp32, which keeps it within the
# 1e-3 bar also where the k-th eigenvalue lies in a near-degenerate bulk
# (gm2000, amp3001; the oracle model of the form measures <= 9e-5 on these
# cases and <= 2e-4 on the coordinates).
EIG_BAR = {"fp64": 1e-10, "fp32": 1e-5, "bf16": 1e-3}
COORD_BAR = {"fp64": 1e-8, "fp32": 1e-3, "bf16": 5e-3, "fp8": 5e-2}
# FP8 (3 fraction bits): Weyl's inequality bounds the move of every
# eigenvalue by the spectral norm of the storage error, |dtheta_i| <=
# ||G_fp8 - G||_2, asserted on every case (the fp8 roundings of G come from
# the oracle's E4M3 model, which is pinned to PyTorch's float8_e4m3fn); the
# 1e-3 relative bar is asserted where the storage error is small against the
# k-th eigenvalue, and amp3001 (k-th eigenvalue in the bulk, 3.5e-3 in the
# oracle model of the form) is reported against it only.
FP8_REL_CASES = {"gm2000_f64", "amp1237_f32", "amp5000_r200"}
# bars against the oracle run with the same storage roundings as the form
# (isolates kernel errors from the precision of the form: what remains is
# fp32 accumulation order and occasional flips of a bf16 rounding)
MATCHED_EIG_BAR = {"fp64": 1e-10, "fp32": 1e-5, "bf16": 1e-4, "fp8": 1e-4, "bf16_all": 1e-4, "fp8_all": 1e-4}


def gm_case(n, dim, comps, var, seed, dtype):
    X, _ = W.gaussian_mixture(n, dim, comps, var, seed)
    return W.euclidean_distances(X, dtype=dtype)


def amp_case(n, refs, seed):
    reads, _ = W.amplicon_reads(n, refs, seed=seed)
    return W.hamming_distances(reads)


CASES = {
    # name: (D builder, k, p, q)
    "gm2000_f64": (lambda: gm_case(2000, 50, 10, 25.0, 0, np.float64), 10, 10, 1),
    "amp1237_f32": (lambda: amp_case(1237, 20, 1), 12, 9, 2),
    "amp3001_f32": (lambda: amp_case(3001, 40, 2), 40, 20, 1),
    # the paper-scale amplicon recipe (200 references, k=100, p=20, q=2) at n=5000
    "amp5000_r200": (lambda: amp_case(5000, 200, 0), 100, 20, 2),
}
_cache = {}


def case(name):
    if name not in _cache:
        build, k, p, q = CASES[name]
        D = build()
        _cache[name] = (D, k, p, q)
    return _cache[name]


def oracle_rand(name, seed=0, keep_history=False, form="fp64"):
    key = (name, seed, keep_history, form)
    if key not in _cache:
        D, k, p, q = case(name)
        _cache[key] = O.rand_mds(D, k, p, q, seed, keep_history=keep_history, form=form)
    return _cache[key]


def fp8_weyl_bound(name):
    """||G_fp8 - G||_2 with G_fp8 the oracle's block-scaled E4M3 operand."""
    key = (name, "weyl")
    if key not in _cache:
        import scipy.sparse.linalg

        D = case(name)[0]
        G = O.gram_matrix(D)
        E = O.fp8_operand(G) - G
        _cache[key] = float(abs(scipy.sparse.linalg.eigsh(0.5 * (E + E.T), k=1, which="LM",
                                                           return_eigenvectors=False)[0]))
    return _cache[key]


def split_sum(X3):
    """x0 + x1 + x2 of a split operand (l_pad x 3 ldg bf16 planes, per 32
    columns the 32 x0, then the x1, then the x2 terms) as l_pad x ldg fp64."""
    X3 = np.asarray(X3, dtype=np.float64)
    ldg = X3.shape[1] // 3
    planes = X3.reshape(X3.shape[0], ldg // 32, 3, 32)
    return (planes[:, :, 0, :] + planes[:, :, 1, :] + planes[:, :, 2, :]).reshape(X3.shape[0], ldg)


def dtype_of(D):
    return "f64" if D.dtype == np.float64 else "f32"


def gpu_run(D, k, p, q, seed, form, **kw):
    plan = mds.Plan(D.shape[0], k, p, q, seed, form=form, d_dtype=dtype_of(D), **kw)
    Dg = torch.from_numpy(np.ascontiguousarray(D)).cuda()
    coords, eig = plan.run(Dg)
    info = plan.info()
    return plan, coords.cpu().numpy(), eig.cpu().numpy(), info


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16", "fp8"])
def test_centring_stage(name, form):
    D, k, p, q = case(name)
    n = D.shape[0]
    say(f"[centring] case={name} n={n} form={form}")
    plan = mds.Plan(n, k, p, q, 0, form=form, d_dtype=dtype_of(D))
    Dg = torch.from_numpy(D).cuda()
    # one range pass: the forms that store no G accumulate ||G||_F^2 and tr G there
    plan.run_stages(Dg, _capi.STAGE_RANGE, 1)
    torch.cuda.synchronize()
    r, c, m = O.centring_stats(D)
    r_g = plan.buffer(_capi.BUF_ROWMEAN).double().cpu().numpy()[:, 0]
    c_g = plan.buffer(_capi.BUF_COLMEAN).double().cpu().numpy()[:, 0]
    m_g = float(plan.buffer(_capi.BUF_MEAN).cpu()[0, 0])
    assert np.max(np.abs(r_g - r) / r) < 1e-13
    assert np.max(np.abs(c_g - c) / c) < 1e-13
    assert abs(m_g - m) / m < 1e-13
    G = O.gram_matrix(D)
    scale = float(np.max(D.astype(np.float64) ** 2))
    if form == "bf16":
        Gg = plan.buffer(_capi.BUF_G).double().cpu().numpy()
        assert np.all(Gg[n:, :] == 0) and np.all(Gg[:, n:] == 0)  # zero padding
        Gg = Gg[:n, :n]
        want = bf16_round(G).astype(np.float64)
        assert (Gg != want).mean() < 1e-4  # only values on a rounding boundary may differ
        assert np.max(np.abs(Gg - G) / np.maximum(np.abs(G), 1e-30 * scale)) <= 2.0 ** -8
    elif form == "fp8":
        codes = plan.buffer(_capi.BUF_G).cpu().double().numpy()  # E4M3 decoded on the host
        sc = plan.buffer(_capi.BUF_GSCALE).cpu().double().numpy()
        assert np.all(codes[n:, :] == 0) and np.all(codes[:, n:] == 0)
        q, s_ref = O.fp8_block_quantize(G)
        assert sc.shape == (-(-n // 256), -(-n // 256))
        s_blk = s_ref[::256, ::256]
        assert np.mean(sc[: s_blk.shape[0], : s_blk.shape[1]] != s_blk) < 1e-2  # equal unless a max sits on a tie
        assert np.mean(codes[:n, :n] != q) < 1e-4
        assert np.all(np.abs(codes) <= 448)
    else:
        with pytest.raises(mds.MdsError):
            plan.buffer(_capi.BUF_G)  # recentred on the fly, never stored
    info = plan.info()
    assert np.isclose(info["sum_sq"], np.sum(D.astype(np.float64) ** 2), rtol=1e-13)
    assert np.isclose(info["frob2"], np.sum(G * G), rtol=1e-11)
    assert np.isclose(info["trace"], np.trace(G), rtol=1e-11, atol=1e-12 * scale)
    assert info["status"] == 0


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("full_stats", [False, True])
def test_centring_trace_nonzero_diagonal(dtype, full_stats):
    # A distance matrix has a zero diagonal, but the centring is defined for any
    # square D: tr G = -1/2 (sum_i d_ii^2 - n m) picks up the diagonal, which lies
    # in several 1024 x 1024 statistics tiles here (n = 2600, ragged last tile).
    # The default statistics read the tiles on and above the diagonal of a
    # symmetric D; full_stats reads all of an asymmetric one (row and column
    # means as written).
    n = 2600
    D, _, _, _ = case("gm2000_f64")
    rng = np.random.default_rng(7)
    Dn = np.abs(rng.standard_normal((n, n))) + 1.0
    Dn[:2000, :2000] = D
    if not full_stats:
        Dn = 0.5 * (Dn + Dn.T)
    Dn[np.arange(n), np.arange(n)] = rng.uniform(0.5, 3.0, n)
    Dn = np.ascontiguousarray(Dn.astype(dtype))
    say(f"[centring trace] n={n} dtype={np.dtype(dtype).name} full_stats={full_stats}")
    plan = mds.Plan(n, 5, 5, 0, 0, form="fp64", d_dtype=dtype_of(Dn), full_stats=full_stats)
    plan.run_stages(torch.from_numpy(Dn).cuda(), _capi.STAGE_RANGE, 1)
    torch.cuda.synchronize()
    G = O.gram_matrix(Dn)
    info = plan.info()
    assert np.isclose(info["trace"], np.trace(G), rtol=1e-12)
    assert np.isclose(info["frob2"], np.sum(G * G), rtol=1e-11)
    D2 = Dn.astype(np.float64) ** 2
    r_g = plan.buffer(_capi.BUF_ROWMEAN).double().cpu().numpy()[:n, 0]
    c_g = plan.buffer(_capi.BUF_COLMEAN).double().cpu().numpy()[:n, 0]
    assert np.allclose(r_g, D2.mean(axis=1), rtol=1e-13, atol=0)
    assert np.allclose(c_g, D2.mean(axis=0), rtol=1e-13, atol=0)


@pytest.mark.parametrize("form", ["fp64", "bf16"])
def test_symmetric_stats_match_full(form):
    # Default statistics (tiles on and above the diagonal, r = c) against the
    # full read on a symmetric D spanning 3 x 3 tiles (n = 3001, ragged last one):
    # the same centring up to the order of the fp64 sums.
    D, k, p, q = case("amp3001_f32")
    n = D.shape[0]
    say(f"[symmetric stats] n={n} form={form}")
    outs = []
    for full in (False, True):
        plan = mds.Plan(n, k, p, q, 0, form=form, d_dtype=dtype_of(D), full_stats=full)
        coords, eig = plan.run(torch.from_numpy(D).cuda())
        torch.cuda.synchronize()
        info = plan.info()
        assert info["status"] == 0, info
        outs.append((eig.cpu().numpy(), info))
        plan.close()
    (e0, i0), (e1, i1) = outs
    for key in ("frob2", "trace", "sum_sq"):
        if key in i0:
            assert np.isclose(i0[key], i1[key], rtol=1e-13), key
    assert np.max(np.abs(e0 - e1)) <= (1e-12 if form == "fp64" else 1e-6) * np.max(np.abs(e1))


@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16", "bf16_all"])
def test_omega_stage(form):
    D, k, p, q = case("amp1237_f32")
    n = D.shape[0]
    seed = 1234567
    l = k + p
    say(f"[omega] n={n} l={l} form={form}")
    plan = mds.Plan(n, k, p, q, seed, form=form.replace("_all", ""), lowp_all_range=form.endswith("_all"))
    plan.run_stages(torch.from_numpy(D).cuda(), _capi.STAGE_OMEGA)
    torch.cuda.synchronize()
    Xt = plan.buffer(_capi.BUF_X).double().cpu().numpy()
    if form == "bf16":  # Omega as the exact three-term split of fl32(Omega); the sketch reads two terms
        Xt = split_sum(Xt)
    Om = O.omega(seed, n, l)
    got = Xt[:l, :n].T
    if form == "fp64":
        # the same IEEE operations in the same order on both sides: bit-identical
        assert np.array_equal(got, Om)
    elif form in ("fp32", "bf16"):
        assert np.max(np.abs(got - Om.astype(np.float32))) <= 2e-7 * np.max(np.abs(Om))
    else:
        assert np.mean(got != bf16_round(Om)) < 1e-3
    assert np.all(Xt[l:, :] == 0) and np.all(Xt[:, n:] == 0)


def test_philox_known_answers_on_device():
    """The device generator's raw blocks against the published known-answer
    vectors of Philox4x64-10, and against the oracle's blocks on the counters
    Omega uses (row i, column block b, key (seed, 0))."""
    from conftest import load_kat

    rows = load_kat("philox4x64_10_kat.txt")
    rng = np.random.default_rng(8)
    extra = [[int(i), int(b), 0, 0, 12345, 0] for i, b in zip(rng.integers(0, 10 ** 6, 500), rng.integers(0, 64, 500))]
    inp = np.array([r[0:6] for r in rows] + extra, dtype=np.uint64)
    say(f"[philox] {len(inp)} blocks on the device")
    din = torch.from_numpy(inp.view(np.int64)).cuda()
    dout = torch.empty((len(inp), 4), dtype=torch.int64, device="cuda")
    st = _capi.lib().mds_philox4x64_10(din.data_ptr(), dout.data_ptr(), len(inp), None)
    assert st == _capi.OK
    torch.cuda.synchronize()
    got = dout.cpu().numpy().view(np.uint64)
    for r, g in zip(rows, got[: len(rows)]):
        assert [int(x) for x in g] == r[6:10]
    want = O.philox4x64_10(inp[len(rows):, :4], (12345, 0))
    assert np.array_equal(got[len(rows):], want)


@pytest.mark.parametrize("name", ["gm2000_f64", "amp1237_f32"])
@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16", "fp8"])
def test_gpass_and_cholqr2_unit(name, form):
    """First G-pass Y = G Omega against an fp64 product of the same rounded
    operands (error bound of recursive summation in the accumulator dtype),
    then CholeskyQR2 of that Y: orthonormal and spanning Y."""
    D, k, p, q = case(name)
    n = D.shape[0]
    l = k + p
    say(f"[gpass] case={name} form={form}")
    plan = mds.Plan(n, k, p, q, 5, form=form, d_dtype=dtype_of(D))
    plan.run_stages(torch.from_numpy(D).cuda(), _capi.STAGE_RANGE, 1)
    torch.cuda.synchronize()
    G = O.gram_matrix(D)
    Om = O.omega(5, n, l)
    # fp32 first pass (fp32 form); the bf16 and fp8 forms take their first
    # range pass with both operands as two-term bfloat16 expansions of their
    # fp32 values (16 significant bits) and three products a0 b0 + a0 b1 +
    # a1 b0: against the exact product of the expansions, the kernel leaves
    # out a1 b1 (below 2^-17 |a b|)
    if form == "fp32":
        G, Om = G.astype(np.float32).astype(np.float64), Om.astype(np.float32).astype(np.float64)
    elif form in ("bf16", "fp8"):
        G, Om = O.round_to(G, "bf16x2"), O.round_to(Om, "bf16x2")
    want = G @ Om
    mag = np.abs(G) @ np.abs(Om)
    Yt = plan.buffer(_capi.BUF_Y).cpu().numpy()
    Y = Yt[:l, :n].T
    u = 2.0 ** -53 if form == "fp64" else 2.0 ** -24
    bound = 2 * n * u * mag
    if form in ("bf16", "fp8"):
        bound = bound + 2.0 ** -16 * mag  # the dropped product a1 b1, and the expansions of nearby fp32 values
    # fp32 passes recentre D on the fly with one fma per entry from fl32(d^2),
    # fl32(c/2), fl32((r-m)/2): a few ulps of those terms (the fused bf16
    # first pass over fp32 D takes fl32 of the fp64 entry itself)
    if form == "fp32" or (form in ("bf16", "fp8") and not (form == "bf16" and D.dtype == np.float32)):
        r, c, m = O.centring_stats(D)
        H = 0.5 * (D.astype(np.float64) ** 2 + c[None, :] + np.abs(r - m)[:, None])
        bound = bound + 4 * u * (H @ np.abs(Om))
    assert np.all(np.abs(Y - want) <= bound + 1e-300)
    assert np.all(Yt[l:] == 0) and np.all(Yt[:, n:] == 0)
    Q = plan.buffer(_capi.BUF_Q).cpu().numpy()[:l, :n].T
    assert np.max(np.abs(Q.T @ Q - np.eye(l))) < 1e-12
    Qy = np.linalg.qr(Y)[0]
    assert span_cos_min(Q, Qy) > 1 - 1e-10


@pytest.mark.parametrize("form", ["bf16", "fp8"])
def test_last_range_pass_unit(form):
    """The last range pass of the low-precision forms, Y = G Q from D with G
    as its two-term bfloat16 expansion and Q rounded once to bfloat16 (two
    products a1 b + a0 b, each exact in fp32), against the fp64 product of
    those rounded operands, Q taken from the device after the pass before."""
    D, k, p, q = case("amp1237_f32")
    n = D.shape[0]
    l = k + p
    say(f"[last pass] form={form} n={n} l={l} q={q}")
    plan = mds.Plan(n, k, p, q, 9, form=form)
    Dg = torch.from_numpy(D).cuda()
    plan.run_stages(Dg, _capi.STAGE_RANGE, 2 * q)
    torch.cuda.synchronize()
    Qp = plan.buffer(_capi.BUF_Q).cpu().numpy()[:l, :n].T
    plan.run_stages(Dg, _capi.STAGE_RANGE, 2 * q + 1)
    torch.cuda.synchronize()
    Yt = plan.buffer(_capi.BUF_Y).cpu().numpy()
    Y = Yt[:l, :n].T
    G = O.gram_matrix(D)
    G2, Qb = O.round_to(G, "bf16x2"), O.round_to(Qp, "bf16")
    want = G2 @ Qb
    mag = np.abs(G2) @ np.abs(Qb)
    u = 2.0 ** -24
    r, c, m = O.centring_stats(D)
    H = 0.5 * (D.astype(np.float64) ** 2 + c[None, :] + np.abs(r - m)[:, None])
    # fp32 accumulation; the kernel's fl32 entries (one fma from fl32(d^2),
    # fl32(c/2), fl32((r-m)/2)) within a few ulps of those terms, and the
    # two-term expansions of such nearby values within 2^-16
    bound = 2 * n * u * mag + 2.0 ** -16 * mag + 4 * u * (H @ np.abs(Qb))
    assert np.all(np.abs(Y - want) <= bound + 1e-300)
    # the operand really is bf16 X: the product with two-term X leaves the bound
    assert np.any(np.abs(Y - G2 @ O.round_to(Qp, "bf16x2")) > bound)
    assert np.all(Yt[l:] == 0) and np.all(Yt[:, n:] == 0)


def test_range_passes_span_fp64():
    name = "gm2000_f64"
    D, k, p, q = case(name)
    ref = oracle_rand(name, keep_history=True)
    plan = mds.Plan(D.shape[0], k, p, q, 0, form="fp64", d_dtype="f64")
    Dg = torch.from_numpy(D).cuda()
    l = k + p
    for passes in range(1, 2 * q + 2):
        say(f"[range] case={name} passes={passes}")
        plan.run_stages(Dg, _capi.STAGE_RANGE, passes)
        torch.cuda.synchronize()
        Qt = plan.buffer(_capi.BUF_Q).cpu().numpy()
        Q = Qt[:l, : D.shape[0]].T
        assert np.max(np.abs(Q.T @ Q - np.eye(l))) < 1e-12
        assert np.all(Qt[l:] == 0)
        assert span_cos_min(Q, ref["history"][passes - 1]) > 1 - 1e-10


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16", "fp8"])
def test_full_run_parity(name, form):
    D, k, p, q = case(name)
    say(f"[full] case={name} form={form}")
    ref = oracle_rand(name)
    matched = oracle_rand(name, form=form)
    plan, X, eig, info = gpu_run(D, k, p, q, 0, form)
    assert info["status"] == 0, info
    err = rel_eig_err(eig, ref["eigvals"])
    merr = rel_eig_err(eig, matched["eigvals"])
    cerr = procrustes_err(X, ref["coords"])
    say(f"    eig rel err vs fp64 {err:.3e}  vs matched {merr:.3e}  coords procrustes {cerr:.3e}"
        f"  fallbacks {info['orth_fallbacks']}  sweeps {info['jacobi_sweeps']}")
    assert merr < MATCHED_EIG_BAR[form]
    assert cerr < COORD_BAR[form]
    if form == "fp8":
        wb = fp8_weyl_bound(name)
        dmax = float(np.max(np.abs(eig - ref["eigvals"])))
        say(f"    fp8: max |dtheta| {dmax:.3e} <= ||G_fp8 - G||_2 = {wb:.3e} (ratio {dmax / wb:.2e})")
        assert dmax <= wb
        if name in FP8_REL_CASES:
            assert err < 1e-3
    else:
        assert err < EIG_BAR[form]
    # theta and V are a Rayleigh-Ritz pair of the projected matrix
    th = plan.buffer(_capi.BUF_THETA).cpu().numpy()[:, 0]
    assert np.all(np.diff(th) <= 0)
    assert np.allclose(th[:k], eig, rtol=0, atol=0)
    # sign convention: largest-magnitude entry of each column is positive
    idx = np.argmax(np.abs(X), axis=0)
    assert np.all(X[idx, np.arange(k)] > 0)
    if form == "fp64":
        assert sign_aligned_err(X, ref["coords"]) < 1e-7


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("form", ["bf16", "fp8"])
def test_lowp_all_range_schedule(name, form):
    """MDS_FLAG_LOWP_ALL_RANGE: every range pass on the stored low-precision G
    (no fp32 end passes).  Checked against the oracle run with that schedule's
    roundings; its error against the plain oracle is reported (it may exceed
    1e-3 where the k-th eigenvalue lies in a near-degenerate bulk)."""
    D, k, p, q = case(name)
    say(f"[lowp all] case={name} form={form}")
    ref = oracle_rand(name)
    matched = oracle_rand(name, form=form + "_all")
    plan = mds.Plan(D.shape[0], k, p, q, 0, form=form, d_dtype=dtype_of(D), lowp_all_range=True)
    coords, eig = plan.run(torch.from_numpy(np.ascontiguousarray(D)).cuda())
    info = plan.info()
    assert info["status"] == 0, info
    eig = eig.cpu().numpy()
    err, merr = rel_eig_err(eig, ref["eigvals"]), rel_eig_err(eig, matched["eigvals"])
    say(f"    eig rel err vs fp64 {err:.3e}  vs matched {merr:.3e}")
    assert merr < MATCHED_EIG_BAR[form + "_all"]


def test_bitwise_repeatable():
    D, k, p, q = case("amp1237_f32")
    say("[repeat] amp1237 bf16 twice")
    plan = mds.Plan(D.shape[0], k, p, q, 3, form="bf16")
    Dg = torch.from_numpy(D).cuda()
    c1, e1 = plan.run(Dg)
    c1, e1 = c1.clone(), e1.clone()
    c2, e2 = plan.run(Dg)
    torch.cuda.synchronize()
    assert torch.equal(c1, c2) and torch.equal(e1, e2)


# ---------------------------------------------------------------------------
# edge cases
def test_zero_distance_matrix():
    n, k, p = 300, 5, 5
    say("[edge] all-zero D")
    D = np.zeros((n, n), dtype=np.float32)
    _, X, eig, info = gpu_run(D, k, p, 1, 0, "fp32")
    assert info["status"] == 0
    assert np.all(eig == 0) and np.all(X == 0)
    assert info["orth_fallbacks"] > 0


def test_nonfinite_input_flagged():
    say("[edge] NaN in D")
    D = amp_case(500, 5, 3)
    D[17, 42] = np.nan
    _, _, _, info = gpu_run(D, 4, 4, 1, 0, "fp32")
    assert info["nonfinite"] == 1 and info["status"] == _capi.ERR_NONFINITE


def test_rank_deficient_matches_exact():
    say("[edge] rank 5 < l = 10")
    X, _ = W.gaussian_mixture(500, 5, 3, 9.0, seed=4)
    D = W.euclidean_distances(X)
    full = O.full_mds(D, 4)
    plan, Xg, eig, info = gpu_run(D, 4, 6, 1, 0, "fp64")
    assert info["status"] == 0
    assert info["orth_fallbacks"] > 0
    assert rel_eig_err(eig, full["eigvals"]) < 1e-10
    assert procrustes_err(Xg, full["coords"]) < 1e-8
    # embedding of an exactly rank-5 cloud with k=4 < 5 keeps G_k = X_k X_k^T
    assert np.allclose(Xg @ Xg.T, full["coords"] @ full["coords"].T, atol=1e-8 * full["eigvals"][0])


def test_rank_deficient_wide_l():
    """l = 150 > 128 on a rank-60 cloud: the factor of the orthonormalisation
    runs as two diagonal blocks and drops columns in both, and the
    eigensolve is the tridiagonal QL; the top 60 eigenpairs are exact."""
    say("[edge] rank 60 < l = 150")
    X, _ = W.gaussian_mixture(700, 60, 5, 9.0, seed=6)
    D = W.euclidean_distances(X)
    full = O.full_mds(D, 60)
    plan, Xg, eig, info = gpu_run(D, 60, 90, 1, 0, "fp64")
    say(f"    fallbacks {info['orth_fallbacks']}, QL steps {info['jacobi_sweeps']}")
    assert info["status"] == 0
    assert info["orth_fallbacks"] > 0
    assert rel_eig_err(eig, full["eigvals"]) < 1e-10
    assert procrustes_err(Xg, full["coords"]) < 1e-8


def test_zero_distance_matrix_wide_l():
    say("[edge] all-zero D, l = 140")
    D = np.zeros((400, 400), dtype=np.float32)
    _, X, eig, info = gpu_run(D, 100, 40, 1, 0, "fp32")
    assert info["status"] == 0
    assert np.all(eig == 0) and np.all(X == 0)
    assert info["orth_fallbacks"] > 0


@pytest.mark.parametrize("k,p,q", [(7, 6, 1), (10, 0, 1), (6, 6, 0), (1, 1, 2)])
def test_shapes_odd_l_no_oversample_no_power(k, p, q):
    say(f"[edge] k={k} p={p} q={q}")
    D = amp_case(777, 15, 5)
    ref = O.rand_mds(D, k, p, q, 9)
    _, X, eig, info = gpu_run(D, k, p, q, 9, "fp64")
    assert info["status"] == 0
    assert rel_eig_err(eig, ref["eigvals"]) < 1e-10
    assert procrustes_err(X, ref["coords"]) < 1e-8


def test_large_l_global_scratch_path():
    say("[edge] l = 140 > 128 (small kernels in global memory)")
    D = amp_case(900, 160, 6)
    k, p, q = 130, 10, 1
    ref = O.rand_mds(D, k, p, q, 2)
    _, X, eig, info = gpu_run(D, k, p, q, 2, "fp64")
    assert info["status"] == 0
    assert rel_eig_err(eig, ref["eigvals"]) < 1e-10
    assert procrustes_err(X, ref["coords"]) < 1e-8


@pytest.mark.parametrize("k,form,full", [(150, "bf16", False), (200, "bf16", False), (200, "bf16", True),
                                         (200, "fp8", False)])
def test_wide_l_streaming_passes(k, form, full):
    """l_pad in (128, 224]: the 16-bit passes from D stream D through LDS with
    up to 14 column groups (fused write and sketch of Omega, last range pass,
    symmetric or full projection), against the oracle with the form's
    roundings and against the plain fp64 method."""
    n, p, q = 3000, 20, 1
    say(f"[wide l] n={n} l={k + p} form={form} full_projection={full}")
    X, _ = W.gaussian_mixture(n, 200, 50, 9.0, 5)
    D = W.euclidean_distances(X, dtype=np.float32)
    ref = O.rand_mds(D, k, p, q, 4, form=form)
    plain = O.rand_mds(D, k, p, q, 4)
    plan = mds.Plan(n, k, p, q, 4, form=form, full_projection=full)
    coords, eig = plan.run(torch.from_numpy(D).cuda())
    info = plan.info()
    torch.cuda.synchronize()
    eig = eig.cpu().numpy()
    err, perr = rel_eig_err(eig, ref["eigvals"]), rel_eig_err(eig, plain["eigvals"])
    say(f"    eig vs matched oracle {err:.2e}, vs plain {perr:.2e}")
    assert info["status"] == 0
    assert err < MATCHED_EIG_BAR[form]
    if form == "bf16":
        assert perr < EIG_BAR["bf16"]
    assert procrustes_err(coords.cpu().numpy(), ref["coords"]) < COORD_BAR[form]


def test_tiny_problem():
    say("[edge] n = 2")
    D = np.array([[0.0, 3.0], [3.0, 0.0]], dtype=np.float32)
    _, X, eig, info = gpu_run(D, 1, 1, 1, 0, "fp64")
    assert info["status"] == 0
    assert np.isclose(eig[0], 4.5, rtol=1e-12)  # G = [[9/4, -9/4], [-9/4, 9/4]]
    assert np.allclose(np.abs(X[:, 0]), 1.5, rtol=1e-12)


def test_d_f64_with_bf16_form():
    name = "gm2000_f64"
    D, k, p, q = case(name)
    say("[dtype] fp64 D, bf16 form")
    ref = oracle_rand(name, form="bf16")
    plain = oracle_rand(name)
    _, X, eig, info = gpu_run(D, k, p, q, 0, "bf16")
    assert info["status"] == 0
    assert rel_eig_err(eig, ref["eigvals"]) < MATCHED_EIG_BAR["bf16"]
    assert rel_eig_err(eig, plain["eigvals"]) < EIG_BAR["bf16"]


# ---------------------------------------------------------------------------
# symmetric projection (default) against the full projection pass
@pytest.mark.parametrize("name", ["gm2000_f64", "amp3001_f32", "amp5000_r200"])
@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16", "fp8"])
@pytest.mark.parametrize("split", [0, 3, 13])
def test_symmetric_projection_matches_full(name, form, split):
    """B assembled from the upper triangle of G equals Q^T G Q from the whole
    of G up to accumulation rounding: same Q (identical range passes), so the
    symmetrised B, the Ritz values and the coordinates must agree closely.
    The bf16/fp8 forms' 16-bit projection splits g_ij and g_ji (which differ
    by the fp32 recentring rounding) separately: their products differ by up
    to 2 2^-15 |g q| more."""
    D, k, p, q = case(name)
    n = D.shape[0]
    say(f"[sym] case={name} form={form} split={split}")
    Dg = torch.from_numpy(np.ascontiguousarray(D)).cuda()
    out = {}
    for full in (False, True):
        plan = mds.Plan(n, k, p, q, 0, form=form, d_dtype=dtype_of(D), gpass_split=split, full_projection=full)
        coords, eig = plan.run(Dg)
        info = plan.info()
        assert info["status"] == 0, info
        B = plan.buffer(_capi.BUF_B).cpu().numpy()
        Q = plan.buffer(_capi.BUF_Q).cpu().numpy()
        out[full] = (coords.cpu().numpy(), eig.cpu().numpy(), 0.5 * (B + B.T), Q)
        plan.close()
    (Xs, es, Bs, Qs), (Xf, ef, Bf, Qf) = out[False], out[True]
    assert np.array_equal(Qs, Qf)  # the range passes do not depend on the projection mode
    l = k + p
    Qn = Qs[:l, :n].T
    G = O.gram_matrix(D)
    u = 2.0 ** -53 if form == "fp64" else 2.0 ** -24
    mag = np.abs(Qn).T @ (np.abs(G) @ np.abs(Qn))
    if form != "fp64":  # recentring terms of the fp32 passes (see the G-pass unit test)
        r, c, m = O.centring_stats(D)
        H = 0.5 * (D.astype(np.float64) ** 2 + c[None, :] + np.abs(r - m)[:, None])
        mag = mag + np.abs(Qn).T @ (H @ np.abs(Qn))
    diff = np.abs(Bs[:l, :l] - Bf[:l, :l])
    bound = (4 * n * u + (2.0 ** -14 if form in ("bf16", "fp8") else 0.0)) * mag
    say(f"    max |B_sym - B_full| / bound {np.max(diff / bound):.3e}, eig rel {rel_eig_err(es, ef):.2e}")
    assert np.all(diff <= bound)
    tol = 1e-12 if form == "fp64" else (1e-5 if form in ("bf16", "fp8") else 1e-6)
    assert rel_eig_err(es, ef) < tol
    assert procrustes_err(Xs, Xf) < (1e-9 if form == "fp64" else 1e-3)


# ---------------------------------------------------------------------------
# projection on bf16 MFMA (two- or three-term split) against fp32 MFMA
@pytest.mark.parametrize("terms", [2, 3])
@pytest.mark.parametrize("name", ["gm2000_f64", "amp1237_f32"])
def test_split_projection_unit(name, terms):
    """The bf16 form's full projection Y = G Q with both operands split into
    bf16 terms: against an fp64 product of the fp32 operands, within the fp32
    pass's bound plus the split's own error per product: 2^-22 for the three
    dropped products of the three-term split (fp32 projection), 2^-15 for the
    two-term one (the default 16-bit projection: each operand within 2^-17,
    a1 b1 dropped)."""
    D, k, p, q = case(name)
    n = D.shape[0]
    l = k + p
    say(f"[split proj] case={name} terms={terms}")
    plan = mds.Plan(n, k, p, q, 3, form="bf16", d_dtype=dtype_of(D), full_projection=True,
                    fp32_projection=terms == 3)
    plan.run(torch.from_numpy(np.ascontiguousarray(D)).cuda())
    assert plan.info()["status"] == 0
    Qt = plan.buffer(_capi.BUF_Q).cpu().numpy()
    Q32 = Qt[:l, :n].T.astype(np.float32).astype(np.float64)
    # the split operand holds fl32(Q) exactly: x0 + x1 + x2 per entry
    recon = split_sum(plan.buffer(_capi.BUF_X).float().cpu().numpy())
    assert np.array_equal(recon[:l, :n], Q32.T)
    assert np.all(recon[l:] == 0) and np.all(recon[:, n:] == 0)
    G = O.gram_matrix(D).astype(np.float32).astype(np.float64)
    want = G @ Q32
    u = 2.0 ** -24
    r, c, m = O.centring_stats(D)
    H = 0.5 * (D.astype(np.float64) ** 2 + c[None, :] + np.abs(r - m)[:, None])
    split_err = 2.0 ** -22 if terms == 3 else 2.0 ** -15
    bound = (2 * n * u + split_err) * (np.abs(G) @ np.abs(Q32)) + 4 * u * (H @ np.abs(Q32))
    Y = plan.buffer(_capi.BUF_Y).cpu().numpy()[:l, :n].T
    say(f"    max |Y - want| / bound {np.max(np.abs(Y - want) / bound):.3e}")
    assert np.all(np.abs(Y - want) <= bound)


@pytest.mark.parametrize("name", ["gm2000_f64", "amp3001_f32", "amp5000_r200"])
@pytest.mark.parametrize("form", ["bf16", "fp8"])
@pytest.mark.parametrize("full", [False, True])
def test_split_projection_matches_fp32_mfma(name, form, full):
    """Same Q, fp32 projection by the three-term split or on fp32 MFMA: B
    agrees within fp32 accumulation bounds, and so do the Ritz values and
    coordinates; the default 16-bit projection (two-term split) agrees with
    them within its own per-product bound, and its Ritz values move by no
    more than the spectral norm of its change of B (Weyl)."""
    D, k, p, q = case(name)
    n = D.shape[0]
    l = k + p
    say(f"[split vs f32] case={name} form={form} full={full}")
    Dg = torch.from_numpy(np.ascontiguousarray(D)).cuda()
    out = {}
    for mode in ("t2", "split", "f32"):
        plan = mds.Plan(n, k, p, q, 0, form=form, d_dtype=dtype_of(D), full_projection=full,
                        fp32_projection=mode == "split", fp32_mfma_projection=mode == "f32")
        coords, eig = plan.run(Dg)
        assert plan.info()["status"] == 0
        B = plan.buffer(_capi.BUF_B).cpu().numpy()
        out[mode] = (coords.cpu().numpy(), eig.cpu().numpy(), 0.5 * (B + B.T), plan.buffer(_capi.BUF_Q).cpu().numpy())
        plan.close()
    (Xs, es, Bs, Qs), (Xf, ef, Bf, Qf), (X2, e2, B2, Q2) = out["split"], out["f32"], out["t2"]
    assert np.array_equal(Qs, Qf) and np.array_equal(Qs, Q2)
    Qn = Qs[:l, :n].T
    G = O.gram_matrix(D)
    r, c, m = O.centring_stats(D)
    H = 0.5 * (D.astype(np.float64) ** 2 + c[None, :] + np.abs(r - m)[:, None])
    mag = np.abs(Qn).T @ ((np.abs(G) + H) @ np.abs(Qn))
    diff = np.abs(Bs[:l, :l] - Bf[:l, :l])
    bound = (4 * n * 2.0 ** -24 + 2.0 ** -21) * mag
    say(f"    max |B_split - B_f32| / bound {np.max(diff / bound):.3e}, eig rel {rel_eig_err(es, ef):.2e}")
    assert np.all(diff <= bound)
    assert rel_eig_err(es, ef) < 1e-6
    assert procrustes_err(Xs, Xf) < 1e-3
    d2 = np.abs(B2[:l, :l] - Bf[:l, :l])
    b2 = (4 * n * 2.0 ** -24 + 2.0 ** -14) * mag
    weyl = np.linalg.norm(B2[:l, :l] - Bf[:l, :l], 2)
    say(f"    16-bit: max |B_t2 - B_f32| / bound {np.max(d2 / b2):.3e}, eig rel {rel_eig_err(e2, ef):.2e}")
    assert np.all(d2 <= b2)
    assert np.max(np.abs(e2 - ef)) <= weyl * (1 + 1e-6) + 1e-12 * np.max(np.abs(ef))
    assert rel_eig_err(e2, ef) < 1e-5


def test_split_fp32_omega():
    """With every fp32 pass split, Omega is written as three bf16 planes whose
    sum is exactly fl32(Omega)."""
    D, k, p, q = case("amp1237_f32")
    n, l, seed = D.shape[0], k + p, 99
    say(f"[split fp32 omega] n={n} l={l}")
    plan = mds.Plan(n, k, p, q, seed, form="fp32", split_fp32=True)
    plan.run_stages(torch.from_numpy(D).cuda(), _capi.STAGE_OMEGA)
    torch.cuda.synchronize()
    recon = split_sum(plan.buffer(_capi.BUF_X).float().cpu().numpy())
    Om = O.omega(seed, n, l).astype(np.float32).astype(np.float64)
    assert np.array_equal(recon[:l, :n], Om.T)
    assert np.all(recon[l:] == 0) and np.all(recon[:, n:] == 0)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("full", [False, True])
def test_split_fp32_form_parity(name, full):
    """The fp32 form with every pass as the three-term bf16 split: same bars as
    the plain fp32 form against the oracle, and agreement with the plain form
    to fp32 rounding."""
    D, k, p, q = case(name)
    say(f"[split fp32] case={name} full={full}")
    ref = oracle_rand(name)
    matched = oracle_rand(name, form="fp32")
    Dg = torch.from_numpy(np.ascontiguousarray(D)).cuda()
    res = {}
    for split in (False, True):
        plan = mds.Plan(D.shape[0], k, p, q, 0, form="fp32", d_dtype=dtype_of(D), split_fp32=split,
                        full_projection=full)
        coords, eig = plan.run(Dg)
        info = plan.info()
        assert info["status"] == 0, info
        res[split] = (coords.cpu().numpy(), eig.cpu().numpy())
        plan.close()
    X, eig = res[True]
    err, merr = rel_eig_err(eig, ref["eigvals"]), rel_eig_err(eig, matched["eigvals"])
    cerr = procrustes_err(X, ref["coords"])
    dplain = rel_eig_err(eig, res[False][1])
    say(f"    eig rel err vs fp64 {err:.3e}  vs matched {merr:.3e}  vs plain fp32 form {dplain:.3e}"
        f"  coords procrustes {cerr:.3e}")
    assert merr < MATCHED_EIG_BAR["fp32"]
    assert err < EIG_BAR["fp32"]
    assert cerr < COORD_BAR["fp32"]
    assert dplain < 1e-6


@pytest.mark.parametrize("form", ["fp32", "bf16", "fp8"])
def test_misaligned_d_matches_aligned(form):
    """D at an address that is not 16-byte aligned takes the per-element load
    paths (and, for the split projection, the register kernel instead of the
    LDS ring): the same sums in the same order, so the results are identical."""
    name = "amp5000_r200"
    D, k, p, q = case(name)
    n = D.shape[0]
    say(f"[misaligned] case={name} form={form}")
    flat = torch.empty(n * n + 1, dtype=torch.float32, device="cuda")
    Dm = flat[1:].view(n, n)
    Dm.copy_(torch.from_numpy(D))
    assert Dm.data_ptr() % 16 != 0
    Da = torch.from_numpy(D).cuda()
    assert Da.data_ptr() % 16 == 0
    res = []
    for Dg in (Da, Dm):
        plan = mds.Plan(n, k, p, q, 0, form=form)
        coords, eig = plan.run(Dg)
        assert plan.info()["status"] == 0
        res.append((coords.cpu().numpy(), eig.cpu().numpy()))
        plan.close()
    assert np.array_equal(res[0][1], res[1][1])
    assert np.array_equal(res[0][0], res[1][0])


# ---------------------------------------------------------------------------
# plan autotuner: the chosen split-K configuration runs and keeps parity
@pytest.mark.parametrize("form", ["fp32", "bf16"])
def test_autotuned_plan_parity(form):
    name = "amp5000_r200"
    D, k, p, q = case(name)
    say(f"[autotune] case={name} form={form}")
    plan = mds.Plan(D.shape[0], k, p, q, 0, form=form)
    Dg = torch.from_numpy(D).cuda()
    r = plan.autotune(Dg)
    say(f"    chosen {r}")
    assert r["candidates"] >= 3 and r["range_ms"] > 0 and r["proj_ms"] > 0
    assert (r["write_ms"] > 0) == (form == "bf16")
    assert (r["f32_ms"] > 0) == (form == "bf16")  # the last range pass of the bf16 form is fp32
    coords, eig = plan.run(Dg)
    info = plan.info()
    assert info["status"] == 0
    if r["range_split"]:
        assert info["gpass_split"] == r["range_split"]
    ref = oracle_rand(name, form=form)
    assert rel_eig_err(eig.cpu().numpy(), ref["eigvals"]) < MATCHED_EIG_BAR[form]
    with pytest.raises(mds.MdsError):
        plan.autotune(Dg)  # the workspace is attached now


# ---------------------------------------------------------------------------
# finite-metric input check (MDS_FLAG_CHECK_INPUT)
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_check_input_flags_asymmetry_and_diagonal(dtype):
    """Symmetric D with a zero diagonal passes; flipped pairs and nonzero
    diagonal entries are counted exactly (several 64 x 64 tiles, ragged
    edge) and the run reports MDS_ERR_NOT_METRIC."""
    n = 1000
    D = amp_case(n, 12, 4).astype(dtype)
    say(f"[check input] n={n} dtype={np.dtype(dtype).name}")
    plan = mds.Plan(n, 5, 5, 1, 0, form="fp64", d_dtype=dtype_of(D), check_input=True)
    plan.run(torch.from_numpy(np.ascontiguousarray(D)).cuda())
    info = plan.info()
    assert info["status"] == 0 and info["asym_pairs"] == 0 and info["diag_nonzero"] == 0
    Db = D.copy()
    pairs = [(3, 900), (64, 65), (999, 0), (500, 501), (10, 11)]
    for i, j in pairs:
        Db[i, j] = Db[i, j] + 0.25  # d_ij != d_ji, one entry per pair
    Db[7, 7] = 0.5
    Db[998, 998] = 1.0
    Db[200, 300] = np.nan  # NaN compares unequal: counted as asymmetric
    plan.run(torch.from_numpy(np.ascontiguousarray(Db)).cuda())
    info = plan.info()
    assert info["asym_pairs"] == len(pairs) + 1 and info["diag_nonzero"] == 2
    assert info["status"] == _capi.ERR_NONFINITE  # non-finite input takes precedence
    Db[200, 300] = Db[300, 200]
    plan.run(torch.from_numpy(np.ascontiguousarray(Db)).cuda())
    info = plan.info()
    assert info["asym_pairs"] == len(pairs) and info["diag_nonzero"] == 2
    assert info["status"] == _capi.ERR_NOT_METRIC
    # without the flag the same D runs through (the contract is not checked)
    plan2 = mds.Plan(n, 5, 5, 1, 0, form="fp64", d_dtype=dtype_of(D))
    plan2.run(torch.from_numpy(np.ascontiguousarray(Db)).cuda())
    assert plan2.info()["status"] == 0
