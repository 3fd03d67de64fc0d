"""CPU tests of the C-ABI library: it loads, exports every declared symbol,
and its host-side logic (parameter derivation, validation, errors) agrees
with the oracle.  No compute calls are made (no GPU here)."""
import os
import re

import numpy as np
import pytest

import oracle
import paper_2201_10132_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tpl_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = _declared("tpl.h")
    assert len(names) >= 20
    L = P.lib()
    for n in names:
        assert hasattr(L, n), n


CASES = [
    dict(nx=64, ny=64, Re=20.0, Wi=0.5, beta=0.8, periods=1),
    dict(nx=1024, ny=1024, Re=60.0, Wi=1.0, beta=0.7, periods=4),
    dict(nx=1024, ny=1024, Re=60.0, Wi=0.0, beta=0.7, periods=4),
    dict(nx=256, ny=256, Re=20.0, Wi=0.5, beta=0.7, periods=4, nq=8, spring=1),
    dict(nx=256, ny=256, Re=20.0, Wi=0.5, beta=0.7, periods=4, nq=8, qe_model=2),
    dict(nx=1024, ny=1024, Re=60.0, Wi=1.0, beta=0.7, periods=4, qe_model=2, tau_drag=0.01,
         tau_ratio_p=0.5),
]


@pytest.mark.parametrize("case", CASES)
def test_derived_parameters_match_oracle(case):
    c = dict(case)
    nq = c.pop("nq", 16)
    spring = c.pop("spring", 0)
    extra = {k: c.pop(k) for k in ("qe_model", "tau_drag", "tau_ratio_p") if k in c}
    t = P.Tpl(c["nx"], c["ny"], c["Re"], c["Wi"], c["beta"], periods=c["periods"], nq=nq,
              spring=spring, **extra)
    o = oracle.OracleSim(1, c["ny"], nq=nq, spring=spring, Re=c["Re"], Wi=c["Wi"],
                         beta=c["beta"], periods=c["periods"], **extra).derived()
    assert t.nqd == oracle.OracleSim(1, 1, nq=nq).nqd
    pairs = dict(kf="kf", l="l", nu="nu", nuS="nuS", G="G", tau1S="tau1S", tau2S="tau2S",
                 tau1P="tau1P", tau2P="tau2P", lambda_eff="lambda", sigma="sigma", R="R",
                 DQ="DQ", F0="F0", kappa="kappa", meq="meq", Sc="Sc")
    for lk, ok in pairs.items():
        assert abs(t.query(lk) - o[ok]) <= 1e-13 * max(1.0, abs(o[ok])), lk


def test_validation_errors():
    with pytest.raises(P.TplError) as e:
        P.Tpl(64, 64, -1.0, 0.5, 0.8)
    assert e.value.code == P.tpl.TPL_EINVAL
    with pytest.raises(P.TplError):
        P.Tpl(64, 64, 20.0, 0.5, 1.5)
    # tau1_S > tau2_S violates the H-theorem ordering
    with pytest.raises(P.TplError) as e:
        P.Tpl(64, 64, 0.01, 0.0, 0.8)
    assert "ordering" in str(e.value)
    t = P.Tpl(64, 64, 20.0, 0.5, 0.8)
    with pytest.raises(P.TplError):
        t.set_param("nq", 7)
    with pytest.raises(P.TplError):
        t.set_param("tau_ratio_p", 1.5)
    with pytest.raises(P.TplError):
        t.set_param("no_such_key", 1)
    with pytest.raises(P.TplError) as e:
        t.step(1)
    assert e.value.code == P.tpl.TPL_ESTATE
    assert P.tpl_last_error()


def test_algorithmic_bytes_formula():
    t = P.Tpl(1024, 1024, 60.0, 1.0, 0.7, periods=4)
    nqd = t.nqd
    N = 1024 * 1024
    # populations read + written, lagged psi written + read, per-node fields
    want = 8 * N * (2 * (9 + 25 * nqd) + 2 * nqd + 2 * 18)
    assert t.query("bytes_per_step") == want


def test_batch_host_logic():
    """Batch creation, validation and parameter forwarding (no device work)."""
    insts = [dict(nx=64, ny=64, Re=20.0, Wi=0.5, beta=0.8),
             dict(nx=32, ny=48, Re=30.0, Wi=1.0, beta=0.7, periods=2, seed=3, perturbation=1e-3)]
    b = P.Batch(insts, nq=8, spring=1)
    assert b.query("instances") == 2
    for i, d in enumerate(insts):
        t = b.instance(i)
        assert (t.query("nx"), t.query("ny")) == (d["nx"], d["ny"])
        assert t.query("nq") == 8 and t.query("spring") == 1
        assert t.query("periods") == d.get("periods", 1)
    want = sum(P.Tpl(d["nx"], d["ny"], d["Re"], d["Wi"], d["beta"], periods=d.get("periods", 1),
                     nq=8).query("bytes_state") for d in insts)
    assert b.query("bytes_state") == want
    with pytest.raises(P.TplError) as e:
        b.set_param("precision", 1)
    assert e.value.code == P.tpl.TPL_EINVAL
    with pytest.raises(P.TplError) as e:
        b.step(1)
    assert e.value.code == P.tpl.TPL_ESTATE
    with pytest.raises(P.TplError):
        b.instance(2)
    with pytest.raises(P.TplError) as e:
        P.Batch([dict(nx=8, ny=8, Re=20.0, Wi=0.5, beta=0.8),
                 dict(nx=8, ny=2, Re=20.0, Wi=0.5, beta=0.8)])
    assert "instance 1" in str(e.value)
    with pytest.raises(P.TplError):
        P.Batch([dict(nx=8, ny=8, Re=20.0, Wi=0.5, beta=0.8)], precision=7)
    b.close()


def test_batched_sweep_draw():
    """The seeded draw of the batched sweep: SplitMix64 pinned to its
    published vectors, values in their ranges, reproducible."""
    from tests import inputs

    path = os.path.join(ROOT, "tests", "golden", "splitmix64_vectors.txt")
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        seed, *outs = [int(v) for v in line.split()]
        g = inputs.splitmix64(seed)
        assert [next(g) for _ in outs] == outs
    c = inputs.c4_instances()
    assert len(c) == 256 and c == inputs.c4_instances()
    assert [d["seed"] for d in c] == list(range(256))
    for d in c:
        assert d["nx"] in inputs.C4_SIZES and d["ny"] in inputs.C4_SIZES
        assert 10 <= d["Re"] < 100 and 0 <= d["Wi"] < 2 and 0.5 <= d["beta"] < 0.9
    # every size appears on both axes
    assert {d["nx"] for d in c} == set(inputs.C4_SIZES) == {d["ny"] for d in c}
    # every instance is a valid configuration for the library
    for d in c[:16]:
        P.Tpl(d["nx"], d["ny"], d["Re"], d["Wi"], d["beta"], periods=d["periods"]).close()


def test_bf16_form_bytes_and_rejections():
    t = P.Tpl(64, 64, 20.0, 0.5, 0.8, nq=8, precision=P.TPL_BF16)
    N, nqd = 64 * 64, t.nqd
    # FP32 solvent and psi, BF16 polymer deviations and the rest population's
    # lower 16 bits (56 bytes per (r, Q))
    assert t.query("bytes_per_step") == N * (2 * 4 * (9 + nqd) + 2 * (2 * 26) * nqd + 16 * 18)
    assert t.query("bytes_XP") == 2 * 2 * 26 * nqd * N
    with pytest.raises(P.TplError):  # null device pointers
        t.adopt_buffers([0, 0, 0, 0], [1, 1, 1, 1])
    with pytest.raises(P.TplError):
        P.Batch([dict(nx=16, ny=16, Re=20.0, Wi=0.5, beta=0.8)], precision=P.TPL_BF16)
    with pytest.raises(P.TplError):
        t.set_param("precision", 3)
    P.Tpl(13, 9, 20.0, 0.5, 0.8, nq=4, precision=P.TPL_BF16).close()  # any node count
    t.close()


def test_tile_group_knobs():
    """Tile-group knobs: launch knobs (settable after init), product of the
    group sides at most 8; the shape in use is 0 before any step."""
    t = P.Tpl(128, 64, 60.0, 1.0, 0.7, periods=2, nq=8)
    with pytest.raises(P.TplError):
        t.set_param("group_x", 16)
    t.set_param("group_x", 4)
    with pytest.raises(P.TplError):
        t.set_param("group_y", 4)  # 16 waves per group
    t.set_param("group_y", 2)
    t.set_param("group_sync", 1)
    t.set_param("autotune", 0)
    assert t.query("group_x") == 4 and t.query("group_y") == 2 and t.query("autotune") == 0
    assert t.query("group_x_used") == 0 and t.query("tune_ms") == 0
    t.close()


def test_qe_model_parameters():
    """Model 2: viscosity from tau2_S, drag time tau1_S = tau_drag (automatic:
    tau2_S) not above tau2_S; Q-diffusivity from tau1_P."""
    t = P.Tpl(256, 256, 20.0, 0.5, 0.8, periods=2, nq=8)
    nuS = t.query("nuS")
    t.set_param("qe_model", 2)  # tau_drag automatic: a BGK solvent
    assert abs(t.query("tau2S") - 3 * nuS) < 1e-15 and t.query("tau1S") == t.query("tau2S")
    t.set_param("tau_drag", 0.5 * t.query("tau2S"))
    assert abs(t.query("DQ") - t.query("tau1P") / 3) < 1e-15
    with pytest.raises(P.TplError):
        t.set_param("tau_drag", 2 * t.query("tau2S"))
    with pytest.raises(P.TplError):
        t.set_param("qe_model", 3)
    t.close()


def test_inplace_storage_knob():
    """In-place streaming: one population array (half the XS and XP bytes,
    same algorithmic bytes per step); FP64 and FP32 only, nx a multiple of
    64, not for batches; population calls need an initialised context."""
    t = P.Tpl(128, 64, 60.0, 1.0, 0.7, periods=2, nq=8)
    two = {k: t.query(k) for k in ("bytes_XS", "bytes_XP", "bytes_PSI", "bytes_FLD",
                                   "bytes_state", "bytes_per_step")}
    t.set_param("inplace", 1)
    assert t.query("inplace") == 1 and t.query("inplace_odd") == 0
    assert t.query("bytes_XS") == two["bytes_XS"] / 2
    assert t.query("bytes_XP") == two["bytes_XP"] / 2
    for k in ("bytes_PSI", "bytes_FLD", "bytes_per_step"):
        assert t.query(k) == two[k]
    assert t.query("bytes_state") == two["bytes_state"] - (two["bytes_XS"] + two["bytes_XP"]) / 2
    t.set_param("precision", P.TPL_FP32)
    with pytest.raises(P.TplError) as e:
        t.set_param("precision", P.TPL_BF16)
    assert e.value.code == P.tpl.TPL_EINVAL
    with pytest.raises(P.TplError):
        t.set_param("inplace", 2)
    with pytest.raises(P.TplError) as e:
        t.get_state()
    assert e.value.code == P.tpl.TPL_ESTATE  # not initialised
    t.close()
    u = P.Tpl(96, 64, 60.0, 1.0, 0.7, periods=2, nq=8)
    with pytest.raises(P.TplError) as e:
        u.set_param("inplace", 1)
    assert "multiple of 64" in str(e.value)
    u.close()
    v = P.Tpl(128, 64, 60.0, 1.0, 0.7, periods=2, nq=8, precision=P.TPL_BF16)
    with pytest.raises(P.TplError):
        v.set_param("inplace", 1)
    v.close()
    b = P.Batch([dict(nx=64, ny=64, Re=20.0, Wi=0.5, beta=0.8)])
    b.set_param("inplace", 1)  # forwarded to every instance
    assert b.instance(0).query("inplace") == 1
    with pytest.raises(P.TplError):
        b.set_param("inplace", 2)
    b.close()
    b = P.Batch([dict(nx=64, ny=64, Re=20.0, Wi=0.5, beta=0.8),
                 dict(nx=96, ny=64, Re=20.0, Wi=0.5, beta=0.8)])
    with pytest.raises(P.TplError) as e:
        b.set_param("inplace", 1)  # an instance whose nx is not a multiple of 64
    assert "multiple of 64" in str(e.value)
    assert b.instance(0).query("inplace") == 0  # the others left as they were
    b.close()


def test_same_step_gradients_knob():
    """Same-step gradients: a parameter before init; its three extra
    launches add a second population read, psi written and read, the
    solvent read and 17 FP64 values per node to the algorithmic bytes."""
    t = P.Tpl(128, 64, 60.0, 1.0, 0.7, periods=2, nq=8)
    N, nqd = 128 * 64, t.nqd
    b0 = t.query("bytes_per_step")
    t.set_param("gradients", 1)
    assert t.query("bytes_per_step") == b0 + N * (200 * nqd + 16 * nqd + 72 + 136)
    with pytest.raises(P.TplError):
        t.set_param("gradients", 2)
    with pytest.raises(P.TplError):
        t.set_param("precision", P.TPL_BF16)
    t.set_param("inplace", 1)  # both together are allowed
    t.close()
    b = P.Batch([dict(nx=64, ny=64, Re=20.0, Wi=0.5, beta=0.8),
                 dict(nx=32, ny=16, Re=20.0, Wi=0.5, beta=0.8)])
    b.instance(1).set_param("spring_shift", 1)
    with pytest.raises(P.TplError):  # the instances' options differ from the batch's
        b.init()
    b.instance(1).set_param("spring_shift", 0)
    b.instance(1).set_param("qe_model", 2)
    b.set_param("gradients", 1)  # forwarded to every instance
    assert [b.instance(i).query("gradients") for i in range(2)] == [1, 1]
    with pytest.raises(P.TplError):  # the instances of a batch share one model
        b.init()
    b.close()


def test_spring_shift_knob():
    t = P.Tpl(128, 64, 60.0, 1.0, 0.7, periods=2, nq=8)
    N, nqd = 128 * 64, t.nqd
    b0 = t.query("bytes_per_step")
    t.set_param("spring_shift", 1)
    assert t.query("bytes_per_step") == b0 + N * (8 * nqd + 16)
    for k, v in (("precision", P.TPL_BF16), ("spring_shift", 2)):
        with pytest.raises(P.TplError):
            t.set_param(k, v)
    # with same-step gradients the M pass is the spring-sum pass: psi read
    # once less and 13 field values per node instead of 17
    t.set_param("gradients", 1)
    assert t.query("bytes_per_step") == b0 + N * (8 * nqd + 16) + N * (200 * nqd + 8 * nqd
                                                                       + 72 + 104)
    t.set_param("inplace", 1)
    t.set_param("precision", P.TPL_FP32)
    t.close()
    b = P.Batch([dict(nx=64, ny=64, Re=20.0, Wi=0.5, beta=0.8)])
    b.set_param("spring_shift", 1)  # forwarded to every instance
    assert b.instance(0).query("spring_shift") == 1
    b.set_param("inplace", 1)
    b.set_param("gradients", 1)
    assert b.instance(0).query("inplace") == 1 and b.instance(0).query("gradients") == 1
    b.close()


def test_batch_model2_rules():
    """A batch runs one quasi-equilibrium model for all its instances, and
    model (ii) with the Taylor form of the spring term; both are checked
    before anything is allocated."""
    from tests import inputs
    b = P.Batch(inputs.c4_instances(2), precision=1, nq=4, pre_steps=10)
    b.instance(1).set_param("qe_model", 2)
    b.instance(1).set_param("tau_drag", 1e-3)
    with pytest.raises(P.TplError) as e:
        b.init()
    assert "qe_model" in str(e.value)
    b.close()
    b = P.Batch(inputs.c4_instances(2), precision=1, nq=4, pre_steps=10, qe_model=2,
                tau_drag=1e-3, spring_shift=1)
    with pytest.raises(P.TplError) as e:
        b.init()
    assert "Taylor" in str(e.value)
    b.close()


def test_health_check_knobs():
    t = P.Tpl(16, 16, 20.0, 0.5, 0.8)
    assert t.query("diag_every") == 0 and t.query("psi_floor") == 1.0
    assert t.query("keep_good") == 0
    t.set_param("diag_every", 5)
    t.set_param("psi_floor", 0.0)
    t.set_param("keep_good", 1)
    assert t.query("diag_every") == 5 and t.query("psi_floor") == 0.0
    assert t.query("keep_good") == 1
    for k, v in (("diag_every", -1), ("psi_floor", -0.5), ("diag_every", 1.5),
                 ("keep_good", 2), ("keep_good", 0.5)):
        with pytest.raises(P.TplError):
            t.set_param(k, v)
    t.close()


def test_init_mode_knob():
    t = P.Tpl(16, 16, 20.0, 0.5, 0.8, spring=1)
    assert t.query("init_mode") == 0
    t.set_param("init_mode", 1)
    with pytest.raises(P.TplError):
        t.set_param("init_mode", 2)
    t.close()
    for kw in (dict(spring=0), dict(spring=1, qe_model=2), dict(spring=1, Wi=0.0)):
        Wi = kw.pop("Wi", 0.5)
        t = P.Tpl(16, 16, 20.0, Wi, 0.8, init_mode=1, **kw)
        with pytest.raises(P.TplError, match="init_mode 1"):  # refused before any device call
            t.init(seed=0, perturbation=0.0)
        t.close()
