"""The packaged selector (paper_2607_12430_amd/selector.bin) against the
method without it, on the first 40 matrices of the selector's evaluation set
(indices 50000-50039 of the selector law: kind, kappa and seed as the law
draws them, SPD at order 4096 and nonsymmetric at order 1024, generated on
the device).  Bounds, fixed before the test was first run:

* every AUTO answer has status ok and a float64 relative residual <= 1e-13;
* AUTO's total time is below that of always-FP32 and of always-BF16SPLIT,
  each escalating to FP64 on failure (the method without the selector), and
  not above that of always-FP64;
* AUTO pays at most half of the failed float factorisations that
  always-FP32 pays (a prediction that a float factor fails sends the input
  to FP64 directly)."""

import pytest

pytestmark = pytest.mark.gpu


def test_selector_gain_on_selector_law():
    from paper_2607_12430_amd import selector
    res = selector.evaluate(selector.DEFAULT_FILE, count=40, first=50_000, n=4096,
                            n_nonsym=1024, kinds=("spd", "nonsym"), device_inputs=True, log=False)
    summary = {k: v for k, v in res.items() if k != "rows"}
    print(summary)
    tot = res["all"]["total_ms"]
    esc = res["all"]["escalations"]
    assert res["auto_all_ok"], [r for r in res["rows"] if not r["auto_ok"]]
    assert tot["auto"] < min(tot["fp32"], tot["bf16split"]), summary
    assert tot["auto"] <= tot["fp64"], summary
    assert esc["auto"] <= esc["fp32"] // 2, summary
