"""CPU checks of the C-ABI library: it loads, exports every symbol of include/hrlb.h, and its
host-side velocity sets (extended-precision discretized Stieltjes) agree with the oracle's
arbitrary-precision tables.  No device work is started here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import quadrature as quad

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "hrlb.h")).read()
    return sorted(set(re.findall(r"\b(hrlb_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_1810_07803_amd import hrlb

    lib = hrlb.load()
    declared = _declared_symbols()
    assert len(declared) >= 18
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(hrlb.EXPORTED)


@pytest.mark.parametrize("Qx,Qy", [(3, 3), (4, 4), (7, 7), (16, 8), (32, 12), (80, 20), (128, 64)])
def test_host_quadrature_matches_oracle_tables(Qx, Qy):
    from paper_1810_07803_amd import hrlb

    q = hrlb.Quadrature(Qx, Qy)
    px, wx, py, wy = q.nodes()
    hr, fr = quad.half_range_rule(Qx), quad.full_range_rule(Qy)
    np.testing.assert_allclose(px[:Qx], hr.nodes_f64(), rtol=4e-16)
    np.testing.assert_allclose(px[Qx:], -hr.nodes_f64(), rtol=4e-16)
    np.testing.assert_allclose(wx[:Qx], hr.weights_f64(), rtol=2e-15)
    np.testing.assert_allclose(py, fr.nodes_f64(), rtol=0, atol=4e-15)
    np.testing.assert_allclose(wy, fr.weights_f64(), rtol=2e-15)


def test_invalid_arguments_are_rejected_with_a_message():
    from paper_1810_07803_amd import hrlb

    with pytest.raises(hrlb.HrlbError) as ei:
        hrlb.Quadrature(2, 4)
    assert ei.value.status == hrlb.HRLB_E_INVALID
    q = hrlb.Quadrature(4, 4)
    for bad in (dict(ncell=31), dict(ncell=6), dict(delta=-1.0), dict(stretch_A=1.0), dict(Tw=0.0)):
        kw = dict(delta=1.0, uw=0.1, ncell=32)
        kw.update(bad)
        with pytest.raises(hrlb.HrlbError) as ei:
            hrlb.workspace_bytes(q, hrlb.make_params(**kw))
        assert ei.value.status == hrlb.HRLB_E_INVALID
        assert len(hrlb.load().hrlb_last_error()) > 0


def test_workspace_size_scales_with_the_state():
    from paper_1810_07803_amd import hrlb

    q = hrlb.Quadrature(16, 8)
    a = hrlb.workspace_bytes(q, hrlb.make_params(delta=0.1, uw=0.2, ncell=512))
    b = hrlb.workspace_bytes(q, hrlb.make_params(delta=0.1, uw=0.2, ncell=512, precision=1))
    units = 512 * 2 * 16 * 8
    assert a > 3 * 2 * units * 8 and b > 3 * 2 * units * 4
    assert a - b >= 3 * 2 * units * 4


def test_kernel_source_digest_ignores_comments_but_not_code():
    # the traffic summaries stay valid across comment edits of the kernel sources and are dropped
    # by any change of the code
    from paper_1810_07803_amd import profiling

    base = 'int a = 1; // note\n/* block\n comment */ const char* s = "x // y";\nfloat f(float v) { return v - -v; }\n'
    same = 'int a = 1;\n// another note\nconst char* s = "x // y";   /* c */\nfloat f(float v) {\n  return v - -v;\n}\n'
    assert profiling.code_only(base) == profiling.code_only(same)
    for changed in (base.replace("1;", "2;"), base.replace('"x // y"', '"x / y"'), base.replace("- -v", "--v")):
        assert profiling.code_only(changed) != profiling.code_only(base)


def test_new_case_parameters_and_empty_batches_are_validated():
    # everything below is rejected on the host, before any device work
    import ctypes as C

    from paper_1810_07803_amd import hrlb

    q = hrlb.Quadrature(4, 4)
    good_table = [(0.5, 0.7, 0.66), (1.0, 1.0, 0.67), (2.0, 1.6, 0.68)]
    assert hrlb.workspace_bytes(q, hrlb.make_params(delta=1.0, uw=0.1, ncell=32, half_channel=1,
                                                    visc_table=good_table, local_dt_cap=64.0)) > 0
    bad = [
        dict(half_channel=2),
        dict(visc_table=good_table[:1]),                                   # one row
        dict(visc_table=[(1.0, 1.0, 0.6)] * 257),                         # too many rows
        dict(visc_table=[(1.0, 1.0, 0.6), (1.0, 1.2, 0.6)]),              # T not increasing
        dict(visc_table=[(-1.0, 1.0, 0.6), (1.0, 1.2, 0.6)]),             # T not positive
        dict(visc_table=[(0.5, 0.0, 0.6), (1.0, 1.2, 0.6)]),              # mu not positive
        dict(visc_table=[(0.5, 1.0, float("nan")), (1.0, 1.2, 0.6)]),     # Pr not finite
        dict(local_dt_cap=-1.0),
        dict(local_dt_cap=2e6),
        dict(ncell=65540),
    ]
    for b in bad:
        kw = dict(delta=1.0, uw=0.1, ncell=32)
        kw.update(b)
        with pytest.raises(hrlb.HrlbError) as ei:
            hrlb.workspace_bytes(q, hrlb.make_params(**kw))
        assert ei.value.status == hrlb.HRLB_E_INVALID, b
    p = hrlb.make_params(delta=1.0, uw=0.1, ncell=32, visc_table=good_table)
    p.visc_mu = None                                                       # NULL row pointer
    with pytest.raises(hrlb.HrlbError):
        hrlb.workspace_bytes(q, p)
    for Qx, Qy in ((129, 4), (4, 65)):
        with pytest.raises(hrlb.HrlbError):
            hrlb.Quadrature(Qx, Qy)
    n = C.c_size_t()
    assert hrlb.load().hrlb_batch_workspace_bytes(None, 0, C.byref(n)) == hrlb.HRLB_E_INVALID


def test_sq_summary_round_trip_and_digest_guard(tmp_path):
    # the SQ-counter summary the profiling helper writes is read back by the benchmark only while the
    # kernel sources keep the digest it records
    import csv

    from paper_1810_07803_amd import profiling

    path = tmp_path / "run_counter_collection.csv"
    cols = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    rows = []
    for disp, kern, valu in ((1, "void hrlb::stage_kernel<float, 1>(args)", 1000.0),
                             (2, "void hrlb::stage_kernel<float, 2>(args)", 3000.0),
                             (3, "void hrlb::stage_kernel<float, 2>(args)", 3000.0)):
        for name, val in (("SQ_INSTS_VALU", valu), ("SQ_INSTS_LDS", 10.0), ("SQ_INSTS_SALU", 5.0)):
            rows.append(dict(Dispatch_Id=disp, Kernel_Name=kern, Counter_Name=name, Counter_Value=val,
                             Start_Timestamp=0, End_Timestamp=1000))
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=cols)
        w.writeheader()
        w.writerows(rows)
    summary = tmp_path / "sq.md"
    summary.write_text(profiling.sq(str(path), 64.0, "cmd"))
    got = profiling.load_sq(str(summary), ["stage_kernel<float, 1>", "stage_kernel<float, 2>"])
    # VALU per unit: wave instructions x 64 lanes / 64 units; weighted by dispatches (1 and 2)
    assert got["valu_per_unit"] == round((1000.0 + 2 * 3000.0) / 3, 1)
    # issue share: instructions x 4 cycles / (1024 SIMDs x 1000 ns x 2.4 GHz)
    assert got["valu_issue_share"] == round((1000.0 * 4 / 2457600 + 2 * 3000.0 * 4 / 2457600) / 3, 3)
    stale = summary.read_text().replace(profiling.source_digest(), "0000000000000000")
    summary.write_text(stale)
    assert profiling.load_sq(str(summary), ["stage_kernel<float, 1>"]) is None


def test_pxy_error_estimate_against_closed_forms():
    # the estimate behind the P_xy error stop rule (host only), against sequences whose remaining error is
    # known in closed form
    import numpy as np

    from paper_1810_07803_amd import hrlb

    L, c = -0.25, 3e-3
    k = np.arange(9)
    # exact geometric decay m_k = L + c r^k (differences d_k = m_{k+1} - m_k, k = 0..7): the fitted rate
    # is r and max(|d_7|, |d_6|) r / (1 - r) = |d_6| r / (1 - r) = c r^7, the remaining error c r^8
    # over r (one check of margin)
    for r in (0.3, 0.7, 0.95):
        m = L + c * r ** k
        assert hrlb.pxy_error_estimate(m) == pytest.approx(c * r ** 7 / abs(m[-1]), rel=1e-9)
        assert hrlb.pxy_error_estimate(m) >= abs(m[-1] - L) / abs(m[-1])
    # alternating decay m_k = L + c (-r)^k: |d| decays at r, |d_6| = c r^6 (1 + r), and the bound is
    # c r^7 (1 + r)/(1 - r), above the remaining error c r^8
    r = 0.6
    m = L + c * (-r) ** k
    assert hrlb.pxy_error_estimate(m) == pytest.approx(c * r ** 7 * (1 + r) / (1 - r) / abs(m[-1]), rel=1e-9)
    # settled: the last two differences exactly zero
    m = np.array([L + 1e-3, L + 1e-4, L + 1e-5, L, L, L])
    assert hrlb.pxy_error_estimate(m) == 0.0
    # not decaying (fitted rate >= 1), or a zero difference inside the window: no estimate
    assert hrlb.pxy_error_estimate(L + 1e-6 * 1.1 ** k) == float("inf")
    m = L + c * 0.5 ** k
    m[3] = m[2]
    assert hrlb.pxy_error_estimate(m) == float("inf")
    with pytest.raises(hrlb.HrlbError):
        hrlb.pxy_error_estimate([L, L])
