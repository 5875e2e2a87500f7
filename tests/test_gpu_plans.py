"""Uneven batching: plans (static and persistent work lists), HIP-graph replay
and the autotuner, all against the oracle and against each other."""
import numpy as np
import pytest

import oracle
from paper_2604_27325_amd import workloads
from tests.parity import compare_batch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2604_27325_amd as bed  # noqa: E402

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def uneven():
    ns, mats = workloads.uneven(batch=1024)
    _, flat = workloads.pack(mats)
    return ns, mats, flat


def run_plan(plan, ns, flat_t):
    lam = torch.empty(int(np.sum(ns)), device=DEV)
    Q = torch.empty_like(flat_t)
    info = torch.empty(len(ns), dtype=torch.int32, device=DEV)
    plan.run(flat_t, lam, Q, info)
    torch.cuda.synchronize()
    return lam, Q, info


def split(ns, lam, Q):
    out_l, out_q, oA, oL = [], [], 0, 0
    for n in ns:
        out_l.append(lam[oL:oL + n])
        out_q.append(Q[oA:oA + n * n].reshape(n, n))
        oA += n * n
        oL += n
    return out_l, out_q


@pytest.mark.parametrize("persistent", [0, 1])
def test_plan_matches_oracle(uneven, persistent):
    ns, mats, flat = uneven
    plan = bed.Plan(torch.float32, ns, tune={"persistent": persistent})
    lam, Q, info = run_plan(plan, ns, torch.from_numpy(flat).to(DEV))
    lam_o, Q_o, _ = oracle.syevd_packed(ns, flat.astype(np.float64))
    lg, qg = split(ns, lam.cpu().numpy(), Q.cpu().numpy())
    lo, qo = split(ns, lam_o, Q_o)
    worst, fails = compare_batch(mats, lg, qg, lo, qo, np.float32, info=info.cpu().numpy())
    print(f"[plan persistent={persistent}] worst {worst}", flush=True)
    assert not fails, fails[:3]


def test_schedules_are_bitwise_identical(uneven):
    """The per-matrix kernel depends only on (n, dtype): static, persistent and
    the convenience path give the same bits, and repeated persistent launches
    (self-resetting work counter) too."""
    ns, mats, flat = uneven
    A = torch.from_numpy(flat).to(DEV)
    outs = []
    for tune in ({"persistent": 0}, {"persistent": 1}, {"persistent": 1, "order": 1}):
        plan = bed.Plan(torch.float32, ns, tune=tune)
        for _ in range(2):
            outs.append(run_plan(plan, ns, A))
    lam_c, Q_c, _ = bed.syevd_packed(ns, A)
    for lam, Q, info in outs:
        assert torch.equal(lam, lam_c) and torch.equal(Q, Q_c)


def test_hip_graph_replay(uneven):
    ns, mats, flat = uneven
    A = torch.from_numpy(flat).to(DEV)
    plan = bed.Plan(torch.float32, ns, tune={"persistent": 1})
    lam = torch.empty(int(np.sum(ns)), device=DEV)
    Q = torch.empty_like(A)
    info = torch.zeros(len(ns), dtype=torch.int32, device=DEV)
    ref_l, ref_q, _ = run_plan(plan, ns, A)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.run(A, lam, Q, info)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run(A, lam, Q, info)
    for rep in range(4):
        lam.fill_(-1.0)
        Q.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _ = (A * 2.0).sum().item()  # eager work between replays
        assert torch.equal(lam, ref_l) and torch.equal(Q, ref_q), f"replay {rep}"


def test_autotune_returns_valid_schedule(uneven):
    ns, mats, flat = uneven
    A = torch.from_numpy(flat).to(DEV)
    lam = torch.empty(int(np.sum(ns)), device=DEV)
    Q = torch.empty_like(A)
    t = bed.autotune(torch.float32, ns, A, lam, Q)
    assert t["threads_big"] in (128, 256, 512) and t["threads_mid"] in (64, 128, 256)
    assert t["leaf"] in (0, 2, 4, 8)
    plan = bed.Plan(torch.float32, ns, tune=t)
    l2, q2, info = run_plan(plan, ns, A)
    lam_o, _, _ = oracle.syevd_packed(ns, flat.astype(np.float64))
    assert np.abs(l2.cpu().numpy() - lam_o).max() <= 1e-5
    assert int(info.abs().sum()) == 0


def test_plan_create_refused_during_capture(uneven):
    ns, _, flat = uneven
    A = torch.from_numpy(flat[: ns[0] * ns[0]]).to(DEV)
    g = torch.cuda.CUDAGraph()
    with pytest.raises(bed.BedError) as ei:
        with torch.cuda.graph(g):
            bed.Plan(torch.float32, [3, 5, 7])
    assert ei.value.status == 5  # BED_ERR_CAPTURE


@pytest.mark.parametrize("persistent", [0, 1])
@pytest.mark.parametrize("big,mid", [(64, 64), (128, 128), (256, 64), (512, 128), (512, 256)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_every_team_shape_matches_oracle(dtype, big, mid, persistent):
    """Every team shape (threads per matrix of the n > 32 and 16 < n <= 32
    classes), including those that accumulate Q_H explicitly on the waves
    outside the reduction, at every n from 1 to 64."""
    rng = np.random.default_rng(3100 + big + mid)
    ns = list(range(1, 65)) + [64, 63, 48, 33, 32, 31, 17, 16, 3]
    mats = [workloads.gaussian_sym(rng, 1, n)[0] for n in ns]
    mats += [workloads.covariance(rng, 1, n)[0] for n in (64, 40, 32, 20)]
    ns += [64, 40, 32, 20]
    _, flat = workloads.pack(mats)
    npdt = np.float32 if dtype == torch.float32 else np.float64
    flat = flat.astype(npdt)
    plan = bed.Plan(dtype, ns, tune={"threads_big": big, "threads_mid": mid,
                                     "persistent": persistent})
    print(f"[shape dtype={dtype} big={big} mid={mid} persistent={persistent}]", flush=True)
    A = torch.from_numpy(flat).to(DEV)
    lam = torch.empty(int(np.sum(ns)), dtype=dtype, device=DEV)
    Q = torch.empty_like(A)
    info = torch.empty(len(ns), dtype=torch.int32, device=DEV)
    plan.run(A, lam, Q, info)
    torch.cuda.synchronize()
    lam_o, Q_o, _ = oracle.syevd_packed(ns, flat.astype(np.float64))
    lg, qg = split(ns, lam.cpu().numpy(), Q.cpu().numpy())
    lo, qo = split(ns, lam_o, Q_o)
    worst, fails = compare_batch(mats, lg, qg, lo, qo, npdt, info=info.cpu().numpy())
    print(f"  worst {worst}", flush=True)
    assert not fails, fails[:3]
    # eigenvalues only (end rows of each node's block carried instead of Q)
    lam_v = torch.empty_like(lam)
    plan.run(A, lam_v, None, info)
    torch.cuda.synchronize()
    lv, _ = split(ns, lam_v.cpu().numpy(), Q.cpu().numpy())
    worst_v, fails_v = compare_batch(mats, lv, None, lo, None, npdt, info=info.cpu().numpy())
    print(f"  eigenvalues only: worst {worst_v}", flush=True)
    assert not fails_v, fails_v[:3]


@pytest.mark.parametrize("leaf", [2, 4, 8])
@pytest.mark.parametrize("big,mid", [(512, 128), (128, 64), (256, 256)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_leaf_cutoff_variants_match_oracle(dtype, big, mid, leaf):
    """Leaves of at most 2, 4 or 8 elements (Sec. 2.2), at every n from 1 to
    64 and on the planted-pair workload (close pairs that deflate), with and
    without eigenvectors."""
    rng = np.random.default_rng(3300 + leaf)
    ns = list(range(1, 65))
    mats = [workloads.gaussian_sym(rng, 1, n)[0] for n in ns]
    for n in (32, 48, 64):
        planted = workloads.paper_scale(n)[0][:8]
        mats += list(planted)
        ns += [n] * len(planted)
    _, flat = workloads.pack(mats)
    npdt = np.float32 if dtype == torch.float32 else np.float64
    flat = flat.astype(npdt)
    plan = bed.Plan(dtype, ns, tune={"threads_big": big, "threads_mid": mid, "leaf": leaf})
    assert plan.tune()["leaf"] == leaf
    print(f"[leaf={leaf} dtype={dtype} big={big} mid={mid}]", flush=True)
    A = torch.from_numpy(flat).to(DEV)
    lam = torch.empty(int(np.sum(ns)), dtype=dtype, device=DEV)
    Q = torch.empty_like(A)
    info = torch.empty(len(ns), dtype=torch.int32, device=DEV)
    plan.run(A, lam, Q, info)
    torch.cuda.synchronize()
    lam_o, Q_o, _ = oracle.syevd_packed(ns, flat.astype(np.float64))
    lg, qg = split(ns, lam.cpu().numpy(), Q.cpu().numpy())
    lo, qo = split(ns, lam_o, Q_o)
    worst, fails = compare_batch(mats, lg, qg, lo, qo, npdt, info=info.cpu().numpy())
    print(f"  worst {worst}", flush=True)
    assert not fails, fails[:3]
    lam_v = torch.empty_like(lam)
    plan.run(A, lam_v, None, info)
    torch.cuda.synchronize()
    lv, _ = split(ns, lam_v.cpu().numpy(), Q.cpu().numpy())
    worst_v, fails_v = compare_batch(mats, lv, None, lo, None, npdt, info=info.cpu().numpy())
    assert not fails_v, fails_v[:3]


def test_uneven_workload_full_size_graph_matches_oracle():
    """The whole uneven workload (4096 matrices, n ~ U{4..64}, spectra
    log-uniform over [1e-4, 1]): autotuned schedule, plan captured in a HIP
    graph, replayed, every matrix against the oracle."""
    ns, mats = workloads.uneven()
    assert len(ns) == 4096
    ns = [int(v) for v in ns]
    _, flat = workloads.pack(mats)
    A = torch.from_numpy(flat).to(DEV)
    lam = torch.empty(int(np.sum(ns)), device=DEV)
    Q = torch.empty_like(A)
    info = torch.zeros(len(ns), dtype=torch.int32, device=DEV)
    tune = bed.autotune(torch.float32, ns, A, lam, Q)
    plan = bed.Plan(torch.float32, ns, tune=tune)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.run(A, lam, Q, info, stream=s)  # warm-up on the capture stream
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.run(A, lam, Q, info, stream=s)
    lam.fill_(-1.0)
    Q.zero_()
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    lam_o, Q_o, _ = oracle.syevd_packed(ns, flat.astype(np.float64))
    lg, qg = split(ns, lam.cpu().numpy(), Q.cpu().numpy())
    lo, qo = split(ns, lam_o, Q_o)
    worst, fails = compare_batch(mats, lg, qg, lo, qo, np.float32, info=info.cpu().numpy())
    print(f"[uneven 4096 graph, schedule {tune}] worst {worst}", flush=True)
    assert not fails, fails[:3]


def test_same_mix_on_two_streams_concurrently():
    """With a persistent schedule stored for a size mix, bed_syevd on two
    streams at once must not share the plan's work counter: each stream's
    result equals the oracle's and the other stream's, bit for bit."""
    ns, mats = workloads.uneven(seed=3200, batch=700)
    ns = [int(v) for v in ns]
    _, flat = workloads.pack(mats)
    bed.tune_set(torch.float32, ns, {"persistent": 1})
    A = torch.from_numpy(flat).to(DEV)
    outs = []
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for st in streams:
        st.wait_stream(torch.cuda.current_stream())
    for rep in range(3):
        pair = []
        for st in streams:
            with torch.cuda.stream(st):
                lam, Q, info = bed.syevd_packed(ns, A, stream=st)
            pair.append((lam, Q, info))
        outs.append(pair)
    torch.cuda.synchronize()
    ref_l, ref_q = outs[0][0][0], outs[0][0][1]
    for pair in outs:
        for lam, Q, info in pair:
            assert torch.equal(lam, ref_l) and torch.equal(Q, ref_q)
            assert int(info.abs().sum()) == 0
    assert bed.cache_entries() >= 2  # one plan per (size mix, stream)
    lam_o, Q_o, _ = oracle.syevd_packed(ns, flat.astype(np.float64))
    lg, qg = split(ns, ref_l.cpu().numpy(), ref_q.cpu().numpy())
    lo, qo = split(ns, lam_o, Q_o)
    worst, fails = compare_batch(mats, lg, qg, lo, qo, np.float32)
    assert not fails, fails[:3]


def test_plan_cache_stays_bounded():
    """More distinct size mixes than the convenience cache holds: it evicts
    (after the evicted plans' launches completed) and every result is right."""
    rng = np.random.default_rng(3300)
    for i in range(40):
        ns = [int(v) for v in rng.integers(3, 40, size=5)] + [i + 2]
        mats = [workloads.gaussian_sym(rng, 1, n)[0].astype(np.float32) for n in ns]
        _, flat = workloads.pack(mats)
        lam, Q, info = bed.syevd_packed(ns, torch.from_numpy(flat).to(DEV))
        assert bed.cache_entries() <= 32
    torch.cuda.synchronize()
    lam_o, _, _ = oracle.syevd_packed(ns, flat.astype(np.float64))
    assert np.abs(lam.cpu().numpy() - lam_o).max() <= 1e-5 * np.abs(lam_o).max()
