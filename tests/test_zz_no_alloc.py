"""The allocation-free entry point bed_syevd_noalloc (work list in the
library's fixed device array) against bed_syevd: two calls in a row on
mixed-size batches, the second smaller, each bitwise equal to bed_syevd (the
same per-matrix kernel configuration) and within the parity rules of the
binary64 oracle; sizes beyond the array's maximum are refused."""
import ctypes

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


def split(ns, lam, Q):
    out_l, out_q, oA, oL = [], [], 0, 0
    for n in ns:
        out_l.append(lam[oL:oL + n])
        out_q.append(Q[oA:oA + n * n].reshape(n, n))
        oA += n * n
        oL += n
    return out_l, out_q


def solve_both(ns, mats):
    _, flat = workloads.pack(mats)
    A = torch.from_numpy(flat).to(DEV)
    lam = torch.full((int(np.sum(ns)),), -7.0, device=DEV)
    Q = torch.full_like(A, -7.0)
    info = torch.full((len(ns),), 99, dtype=torch.int32, device=DEV)
    bed.syevd_noalloc_packed(ns, A, lam, Q, info)
    lam_r, Q_r, info_r = bed.syevd_packed(ns, A)
    torch.cuda.synchronize()
    assert torch.equal(lam, lam_r) and torch.equal(Q, Q_r) and torch.equal(info, info_r)
    lam_o, Q_o, _ = oracle.syevd_packed(ns, flat.astype(np.float64))
    lg, qg = split(ns, lam.cpu().numpy(), Q.cpu().numpy())
    lo, qo = split(ns, lam_o, Q_o)
    worst, fails = compare_batch(mats, lg, qg, lo, qo, np.float32, info=info.cpu().numpy())
    print(f"[noalloc batch {len(ns)}] worst {worst}", flush=True)
    assert not fails, fails[:3]


def test_noalloc_matches_syevd_two_calls():
    ns, mats = workloads.uneven(seed=3100, batch=2500)  # two list chunks
    solve_both([int(v) for v in ns], mats)
    ns2, mats2 = workloads.uneven(seed=3101, batch=300)  # smaller: stale items must not matter
    solve_both([int(v) for v in ns2], mats2)


def test_noalloc_uniform_and_limits():
    rng = np.random.default_rng(3102)
    A = torch.from_numpy(workloads.gaussian_sym(rng, 40, 24).astype(np.float32)).to(DEV)
    lam = torch.empty(40 * 24, device=DEV)
    Q = torch.empty(40 * 24 * 24, device=DEV)
    bed.syevd_noalloc_packed([24] * 40, A.view(-1), lam, Q)
    lam_r, Q_r = bed.syevd(A)
    assert torch.equal(lam, lam_r.view(-1)) and torch.equal(Q, Q_r.view(-1))
    lib = bed.load_library()
    big = np.full(65537, 3, dtype=np.int32)
    x = torch.empty(65537 * 9, device=DEV)
    st = lib.bed_syevd_noalloc(0, len(big), big.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                               ctypes.c_void_p(x.data_ptr()), None, None)
    assert st == 1  # BED_ERR_INVALID_ARG: beyond the fixed array
