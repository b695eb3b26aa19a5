"""C ABI checks that need no GPU: the library loads, exports every declared symbol, and
rejects bad arguments before touching the HIP runtime."""
import ctypes

import pytest

import paper_2602_02500_amd as ifn


@pytest.fixture(scope="module")
def L():
    return ifn.load()


def test_exports_every_header_symbol(L):
    names = ifn.header_functions()
    assert len(names) >= 8
    for n in names:
        assert hasattr(L, n), n


def _plan(L, exps, coeffs, basis=0, norm=0, compute=1, mode=0, flags=0, rows=(64,), cols=(96,), ind=1, outd=1):
    K = len(exps)
    e = (ctypes.c_int32 * max(K, 1))(*exps)
    c = (ctypes.c_double * max(K, 1))(*coeffs)
    d = ifn.PolyDesc(K, e, c, basis, norm, compute, mode, None, 0, flags)
    n = len(rows)
    r = (ctypes.c_int64 * n)(*rows)
    cc = (ctypes.c_int64 * n)(*cols)
    h = ctypes.c_void_p()
    st = L.ifnso_plan(ctypes.byref(d), n, r, cc, ind, outd, 0, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("exps,coeffs", [
    ([3], [1.0]),               # not a power of two
    ([0, 2, 1], [1, 1, 1]),     # not increasing
    ([0, 0], [1, 1]),           # repeated
    ([1 << 16], [1.0]),         # above 2^15
    ([-1], [1.0]),
    ([], []),                   # no terms
    ([0, 1], [1.0, float("nan")]),
])
def test_plan_rejects_bad_polynomials(L, exps, coeffs):
    st, _ = _plan(L, exps, coeffs)
    assert st == 1, L.ifnso_last_error()


def test_plan_rejects_bad_enums_and_shapes(L):
    assert _plan(L, [0, 1], [1, 1], basis=7)[0] == 1
    assert _plan(L, [0, 1], [1, 1], norm=9)[0] == 1
    assert _plan(L, [0, 1], [1, 1], compute=5)[0] == 1
    assert _plan(L, [0, 1], [1, 1], rows=(0,))[0] == 1
    assert _plan(L, [0, 1], [1, 1], cols=(-3,))[0] == 1
    assert _plan(L, [0, 1], [1, 1], ind=4)[0] == 1


def test_sum_one_flag(L):
    st, _ = _plan(L, [0, 1], [0.5, 0.6], flags=ifn.FLAG_ENFORCE_SUM_ONE)
    assert st == 1 and b"sum" in L.ifnso_last_error()


def test_split_flag_requirements(L):
    """Split bf16 operands are a complement-basis, bf16-compute, fixed-coefficient option."""
    split = ifn.FLAG_SPLIT_BF16
    assert _plan(L, [0, 1, 2], [1, 1, 1], basis=0, compute=1, flags=split)[0] == 1  # Gram basis
    assert b"SPLIT" in L.ifnso_last_error()
    assert _plan(L, [0, 1, 2], [1, 1, 1], basis=1, compute=0, flags=split)[0] == 1  # float32 compute
    assert _plan(L, [0, 1, 2], [1, 1, 1], basis=1, compute=2, flags=split)[0] == 1  # e4m3 compute
    assert _plan(L, [0, 1, 2], [1, 1, 1], basis=1, compute=1, flags=16)[0] == 1     # unknown bit


def test_flag_values_and_split_p_requirements(L):
    """The flag bits of the C ABI; split P is a Gram-basis, bf16-compute, fixed-coefficient
    option that needs a squaring; the deterministic flag is accepted everywhere."""
    import re
    hdr = open(ifn.HEADER_PATH).read()
    for name, val in (("ENFORCE_SUM_ONE", 1), ("DETERMINISTIC", 2), ("SPLIT_P", 4), ("SPLIT_BF16", 8)):
        assert re.search(r"IFNSO_FLAG_%s = %d\b" % (name, val), hdr), name
        assert getattr(ifn, "FLAG_" + name) == val
    sp = ifn.FLAG_SPLIT_P
    assert _plan(L, [0, 1, 2], [1, 1, 1], basis=1, compute=1, flags=sp)[0] == 1      # complement basis
    assert b"SPLIT_P" in L.ifnso_last_error()
    assert _plan(L, [0, 1, 2], [1, 1, 1], basis=0, compute=0, flags=sp)[0] == 1      # float32 compute
    assert _plan(L, [0, 1, 2], [1, 1, 1], basis=0, compute=2, flags=sp)[0] == 1      # e4m3 compute
    assert _plan(L, [0, 1], [1.5, -0.5], basis=0, compute=1, flags=sp)[0] == 2       # no squaring
    for compute, basis in ((0, 0), (1, 0), (1, 1), (2, 0)):  # accepted: fails later only at the device
        ind = ifn.F32 if compute == 0 else ifn.BF16
        st, _ = _plan(L, [0, 1, 2], [0.5, 0.25, 0.25], basis=basis, compute=compute, flags=ifn.FLAG_DETERMINISTIC,
                      ind=ind, outd=ind)
        assert st in (0, 4), L.ifnso_last_error()


def test_unsupported_combinations(L):
    assert _plan(L, [0, 1], [1, 1], compute=ifn.COMPUTE_F32, ind=ifn.BF16)[0] == 2
    assert _plan(L, [0, 1], [1, 1], compute=ifn.COMPUTE_BF16, ind=ifn.F32)[0] == 2
    assert _plan(L, [0, 1], [1, 1], mode=1)[0] == 1  # learned mode without parameters


def test_fp8_requirements(L):
    fp8 = ifn.COMPUTE_FP8
    assert _plan(L, [0, 1, 2], [0.5, 0.25, 0.25], basis=1, compute=fp8)[0] == 2   # complement basis
    assert _plan(L, [0, 1, 2], [0.5, 0.25, 0.25], compute=fp8, ind=ifn.F32)[0] == 2  # float32 input
    # h * round_up(w, 16) must stay below 2^31 (checked before the device is touched)
    assert _plan(L, [0, 1, 2], [0.5, 0.25, 0.25], compute=fp8, rows=(32000,), cols=(1 << 17,))[0] == 2


def test_quantize_e4m3_argument_checks(L):
    need = L.ifnso_quantize_e4m3_workspace_bytes(64, 100)
    assert need > 0 and L.ifnso_quantize_e4m3_workspace_bytes(0, 100) == 0
    # M at 4096 (64 x 100 bf16), Q at 1 << 20, out3 at 1 << 24, workspace at 1 << 25
    q = lambda **k: L.ifnso_quantize_e4m3(k.get("M", 4096), 64, 100, k.get("ldm", 100), k.get("Q", 1 << 20),
                                          k.get("ldq", 112), k.get("out", 1 << 24), 1 << 25, k.get("nb", need), None)
    assert q(M=None) == 1
    assert q(out=None) == 1
    assert q(ldm=99) == 1            # ldm < cols
    assert q(ldq=100) == 1           # below round_up(100, 16)
    assert q(ldq=120) == 1           # not a multiple of 16
    assert q(Q=(1 << 20) + 8) == 1   # Q not 16-byte aligned
    assert q(Q=4096 + 64) == 1       # Q overlaps M
    assert q(nb=need - 1) == 3
    assert L.ifnso_quantize_e4m3(4096, 64, 100, 100, 1 << 20, 1 << 26, 1 << 24, 1 << 25, need, None) == 2


def test_learned_mode_requirements(L):
    params = (ctypes.c_float * ifn.MLP_NUM_PARAMS)(*([0.0] * ifn.MLP_NUM_PARAMS))

    def plan(exps, basis=0, norm=0, compute=1, n=ifn.MLP_NUM_PARAMS):
        e = (ctypes.c_int32 * len(exps))(*exps)
        c = (ctypes.c_double * len(exps))(*([1.0 / len(exps)] * len(exps)))
        d = ifn.PolyDesc(len(exps), e, c, basis, norm, compute, 1, params, n, 0)
        r = (ctypes.c_int64 * 1)(64)
        cc = (ctypes.c_int64 * 1)(96)
        h = ctypes.c_void_p()
        return L.ifnso_plan(ctypes.byref(d), 1, r, cc, 1 if compute else 0, 1 if compute else 0, 0, ctypes.byref(h))

    assert plan([0, 1, 2, 4, 8]) == 2                     # other exponents: not predicted
    assert plan([0, 1, 2, 4, 8, 16], basis=1) == 2        # complement basis
    assert plan([0, 1, 2, 4, 8, 16], norm=1) == 2
    assert plan([0, 1, 2, 4, 8, 16], compute=0) == 2      # float32 compute
    assert plan([0, 1, 2, 4, 8, 16], compute=2) == 2      # e4m3 compute
    assert plan([0, 1, 2, 4, 8, 16], n=100) == 1          # wrong parameter count
    params[7] = float("inf")
    assert plan([0, 1, 2, 4, 8, 16]) == 1                 # non-finite parameter
    params[7] = 0.0


def test_mlp_entry_points_reject_bad_arguments(L):
    assert L.ifnso_mlp_features(0, 16, 16, 8, 16, None) == 1
    assert L.ifnso_mlp_forward(1, None, 16, 16, None) == 1
    assert L.ifnso_mlp_train_workspace_bytes(0) == 0
    need = L.ifnso_mlp_train_workspace_bytes(4)
    assert need >= 4 * ifn.MLP_NUM_PARAMS * 4
    args = [4, 16, 16, 16, 8, 16, 16, 16, 1, 1e-3, 0.9, 0.999, 1e-8, None, None]
    assert L.ifnso_mlp_train_step(*args, 256, need - 1, None) == 3
    bad = list(args)
    bad[10] = 1.5  # beta1 outside [0, 1)
    assert L.ifnso_mlp_train_step(*bad, 256, need, None) == 1
    bad = list(args)
    bad[8] = 0  # step number
    assert L.ifnso_mlp_train_step(*bad, 256, need, None) == 1


def test_null_arguments(L):
    h = ctypes.c_void_p()
    assert L.ifnso_plan(None, 1, None, None, 1, 1, 0, ctypes.byref(h)) == 1
    assert L.ifnso_plan_destroy(None) == 0
    assert L.ifnso_orthogonalize(None, None, 0, None, 0, None, 0, None) == 1
    sz = ctypes.c_size_t()
    assert L.ifnso_plan_workspace_bytes(None, ctypes.byref(sz)) == 1


def test_classical_ns_argument_checks(L):
    abc = (ctypes.c_double * 3)(3.4445, -4.775, 2.0315)
    assert L.ifnso_classical_ns(None, 4, 4, 4, 0, 16, 4, 5, abc, 0, 256, 1 << 20, None) == 1
    assert L.ifnso_classical_ns(1024, 4, 8, 4, 0, 4096, 8, 5, abc, 0, 256, 1 << 20, None) == 1  # ldm < cols
    assert L.ifnso_classical_ns(1024, 4, 8, 8, 0, 4096, 8, 0, abc, 0, 256, 1 << 20, None) == 1  # steps
    assert L.ifnso_classical_ns(1024, 4, 8, 8, 0, 4096, 8, 2, abc, 1, 256, 1 << 20, None) == 2  # f32 data, bf16 compute
    need = L.ifnso_classical_ns_workspace_bytes(4, 8, 0)
    assert need > 0
    assert L.ifnso_classical_ns(1024, 4, 8, 8, 0, 1 << 30, 8, 2, abc, 0, 256, need - 1, None) == 3
    assert L.ifnso_classical_ns(1024, 4, 8, 8, 0, 1028, 8, 2, abc, 0, 256, need, None) == 1  # overlap
    assert L.ifnso_classical_ns_workspace_bytes(0, 8, 0) == 0


def test_ns_schedule_argument_checks(L):
    n = 17
    abc = (ctypes.c_double * (3 * n))(*([3.4445, -4.775, 2.0315] * n))
    need = L.ifnso_classical_ns_workspace_bytes(4, 8, 0)
    args = lambda steps, q, ws=need: (1024, 4, 8, 8, 0, 1 << 30, 8, steps, abc, q, 0, 256, ws, None)
    assert L.ifnso_ns_schedule(*args(0, 0)) == 1  # no steps
    assert L.ifnso_ns_schedule(*args(17, 0)) == 1  # more than IFNSO_NS_MAX_STEPS
    assert L.ifnso_ns_schedule(*args(3, -1)) == 1  # negative q
    assert L.ifnso_ns_schedule(*args(3, 3)) == 2  # q above 2 not built
    assert L.ifnso_ns_schedule(*args(3, 2, need - 1)) == 3
    assert L.ifnso_ns_schedule(1024, 4, 8, 8, 0, 1 << 30, 8, 3, None, 0, 0, 256, need, None) == 1
    bad = (ctypes.c_double * 6)(1.0, 0.0, 0.0, float("nan"), 0.0, 0.0)
    assert L.ifnso_ns_schedule(1024, 4, 8, 8, 0, 1 << 30, 8, 2, bad, 0, 0, 256, need, None) == 1
    assert b"finite" in L.ifnso_last_error()
    # the header's step bound
    with open(ifn.HEADER_PATH) as f:
        assert "#define IFNSO_NS_MAX_STEPS 16" in f.read()


def test_workspace_sizes_grow_with_shape(L):
    a = L.ifnso_classical_ns_workspace_bytes(256, 512, 1)
    b = L.ifnso_classical_ns_workspace_bytes(1024, 4096, 1)
    c = L.ifnso_classical_ns_workspace_bytes(4096, 1024, 1)
    assert 0 < a < b and b == c
    assert L.ifnso_orth_error_workspace_bytes(0) == 0
    assert L.ifnso_orth_error_workspace_bytes(224) > 224 * 32


def test_stage_config_argument_checks(L):
    c = ifn.StageConfig(1, 32, 4, 8, 32)
    assert L.ifnso_plan_get_config(None, 0, ctypes.byref(c)) == 1
    assert L.ifnso_plan_set_config(None, 0, ctypes.byref(c)) == 1


def test_c_client_compiles_and_links(tmp_path):
    """The plain-C client of the ABI builds with gcc against include/ifnso.h and libifnso.so
    alone; without a GPU it stops after its device check."""
    import subprocess
    import __graft_entry__ as ge
    exe = ge.build_capi_client(str(tmp_path / "capi_client"))
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode in (0, 2), r.stdout + r.stderr
    assert ("no GPU" in r.stdout) or r.stdout.strip().endswith("OK")


def test_binding_rejects_mismatched_tensors():
    """The binding checks every tensor against the plan before any pointer reaches the C ABI:
    dtype, shape, row-major layout with unit column stride, device, and for workspaces size,
    contiguity and alignment. On the CPU the device check is the last one to fire."""
    import torch
    shape = (6, 10)
    good = torch.zeros(shape, dtype=torch.bfloat16)
    with pytest.raises(TypeError):
        ifn.check_matrix(good.float(), "M", shape, ifn.BF16, 0)
    with pytest.raises(TypeError):
        ifn.check_matrix(good, "Y", shape, ifn.F32, 0)
    with pytest.raises(TypeError):
        ifn.check_matrix([1.0], "M", shape, ifn.BF16, 0)
    with pytest.raises(ValueError):
        ifn.check_matrix(torch.zeros((6, 11), dtype=torch.bfloat16), "M", shape, ifn.BF16, 0)
    with pytest.raises(ValueError):
        ifn.check_matrix(torch.zeros((60,), dtype=torch.bfloat16), "M", shape, ifn.BF16, 0)
    with pytest.raises(ValueError):  # a column-strided view: every other element
        ifn.check_matrix(torch.zeros((6, 20), dtype=torch.bfloat16)[:, ::2], "M", shape, ifn.BF16, 0)
    with pytest.raises(ValueError):  # a transposed view (column-major)
        ifn.check_matrix(torch.zeros((10, 6), dtype=torch.bfloat16).t(), "M", shape, ifn.BF16, 0)
    with pytest.raises(ValueError) as e:  # every other property holds: the device is wrong
        ifn.check_matrix(good, "M", shape, ifn.BF16, 0)
    assert "cuda:0" in str(e.value)
    # a row-padded view (leading dimension above the column count) is a valid layout
    padded = torch.zeros((6, 16), dtype=torch.bfloat16)[:, :10]
    with pytest.raises(ValueError) as e:
        ifn.check_matrix(padded, "M", shape, ifn.BF16, 0)
    assert "cuda:0" in str(e.value)


def test_binding_rejects_bad_workspaces():
    import torch
    with pytest.raises(TypeError):
        ifn.check_workspace(12345, 64, 0)
    with pytest.raises(ValueError):
        ifn.check_workspace(torch.empty(63, dtype=torch.uint8), 64, 0)
    with pytest.raises(ValueError):
        ifn.check_workspace(torch.empty((16, 8), dtype=torch.uint8).t(), 64, 0)
    with pytest.raises(ValueError) as e:
        ifn.check_workspace(torch.empty(64, dtype=torch.uint8), 64, 0)
    assert "cuda:0" in str(e.value)


def test_schedule_plan_argument_checks(L):
    """ifnso_schedule_plan refuses bad arguments before touching the device."""
    def mk(abc, steps, q=0, rows=(64,), cols=(96,), dtype=1, compute=1):
        a = (ctypes.c_double * max(len(abc), 1))(*abc)
        n = len(rows)
        r = (ctypes.c_int64 * n)(*rows)
        c = (ctypes.c_int64 * n)(*cols)
        h = ctypes.c_void_p()
        return L.ifnso_schedule_plan(a, steps, q, n, r, c, dtype, compute, 0, ctypes.byref(h))
    muon = [3.4445, -4.775, 2.0315]
    assert mk(muon, 0) == 1                      # no steps
    assert mk(muon * 17, 17) == 1                # beyond IFNSO_NS_MAX_STEPS
    assert mk(muon, 1, q=-1) == 1
    assert mk(muon, 1, q=2) == 2                 # Gelfand q = 2 is single-matrix only
    assert mk([1.0, float("inf"), 0.0], 1) == 1
    assert mk(muon, 1, dtype=7) == 1
    assert mk(muon, 1, rows=(0,)) == 1
    assert L.ifnso_schedule_plan(None, 1, 0, 1, None, None, 1, 1, 0, None) == 1
    assert L.ifnso_schedule_orthogonalize_batched(None, None, None, None, None, None, 0, None) == 1
    assert L.ifnso_schedule_plan_destroy(None) == 0
