"""The C ABI library loads and exports every entry point its header declares
(no device calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def _declared():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(pphd_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_paper_stages():
    names = _declared()
    for n in ("pphd_predict", "pphd_update", "pphd_extract", "pphd_resample", "pphd_exchange",
              "pphd_create", "pphd_init", "pphd_destroy", "pphd_workspace_size", "pphd_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1503_03769_amd import pphd
    L = ctypes.CDLL(pphd.LIB_PATH)
    for n in _declared():
        assert hasattr(L, n), n
    # the binding wraps every declared entry point under the same name
    for n in _declared():
        assert n in pphd.SIGNATURES, n
        assert hasattr(pphd, n), n


def test_workspace_size_and_argument_errors():
    """pphd_workspace_size is pure host arithmetic: check it and its error path."""
    from paper_1503_03769_amd import pphd
    from paper_1503_03769_amd.scenario import WORKLOADS
    w = WORKLOADS["large_fp32_10tgt_k64"]
    m = pphd.model_struct(w["model"], pphd.PPHD_FP32)
    n32 = pphd.pphd_workspace_size(m, w["cap"], w["max_meas"])
    m64 = pphd.model_struct(w["model"], pphd.PPHD_FP64)
    n64 = pphd.pphd_workspace_size(m64, w["cap"], w["max_meas"])
    KC = 64 * w["cap"]
    assert n32 >= 2 * 5 * KC * 4 and n64 >= 2 * 5 * KC * 8 and n64 > n32
    bad = pphd.model_struct(dict(w["model"], partitions=0), pphd.PPHD_FP32)
    with pytest.raises(pphd.PphdError) as e:
        pphd.pphd_workspace_size(bad, w["cap"], w["max_meas"])
    assert e.value.code == pphd.PPHD_EINVAL
    with pytest.raises(pphd.PphdError):
        pphd.pphd_workspace_size(m, 10, w["max_meas"])          # cannot hold round(R/K)
    with pytest.raises(pphd.PphdError):
        pphd.pphd_workspace_size(m, w["cap"], 0)
    assert pphd.pphd_kernel_name(3) == "k_weight"
    assert [pphd.pphd_kernel_name(i) for i in range(pphd.K_COUNT)][-5:] == ["k_mlp_infer", "k_birth_mix", "k_zprep", "k_bk_scatter", "k_bk_back"]
    assert pphd.pphd_kernel_name(pphd.K_COUNT) is None


def test_learned_proposal_declarations_and_config_errors():
    from paper_1503_03769_amd import pphd
    names = _declared()
    for n in ("pphd_mlp_create", "pphd_mlp_train", "pphd_mlp_loss_grad", "pphd_mlp_forward",
              "pphd_attach_mlp", "pphd_set_birth_mixture"):
        assert n in names
    ok = pphd.pphd_mlp_config(4096, 1 << 20, 1e-3, 0.9, 0.999, 1e-8)
    n = pphd.pphd_mlp_workspace_size(ok)
    # the dataset (6 floats per pair) and one gradient partial per 64-pair tile
    assert n >= (1 << 20) * 24 + 64 * 38052 * 4
    for bad in (pphd.pphd_mlp_config(100, 1 << 20, 1e-3, 0.9, 0.999, 1e-8),
                pphd.pphd_mlp_config(4096, 5000, 1e-3, 0.9, 0.999, 1e-8),
                pphd.pphd_mlp_config(4096, 8192, -1.0, 0.9, 0.999, 1e-8)):
        with pytest.raises(pphd.PphdError):
            pphd.pphd_mlp_workspace_size(bad)


def test_global_cz_argument_checks():
    """The global-C reading is 0 or 1, and a batch using it needs every run
    to have the same partition count (the split masses use one K)."""
    from paper_1503_03769_amd import pphd
    from paper_1503_03769_amd.scenario import BASE_MODEL
    assert pphd.pphd_workspace_size(pphd.model_struct(dict(BASE_MODEL, partitions=4, global_cz=1), pphd.PPHD_FP32),
                                    4000, 64) > 0
    with pytest.raises(pphd.PphdError) as e:
        pphd.pphd_workspace_size(pphd.model_struct(dict(BASE_MODEL, partitions=4, global_cz=2), pphd.PPHD_FP32),
                                 4000, 64)
    assert e.value.code == pphd.PPHD_EINVAL
    runs = [dict(partitions=4, births_per_step=800, clutter_rate=10.0, particles_per_target=2000.0, run_id=0),
            dict(partitions=2, births_per_step=800, clutter_rate=10.0, particles_per_target=2000.0, run_id=1)]
    t = pphd.run_table(runs)
    for gz, ok in ((0, True), (1, False)):
        m = pphd.model_struct(dict(BASE_MODEL, partitions=1, global_cz=gz), pphd.PPHD_FP32)
        if ok:
            assert pphd.pphd_batch_workspace_size(m, ctypes.addressof(t), 2, 2048, 64) > 0
        else:
            with pytest.raises(pphd.PphdError):
                pphd.pphd_batch_workspace_size(m, ctypes.addressof(t), 2, 2048, 64)
