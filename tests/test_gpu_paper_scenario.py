"""The paper's accuracy comparison in its own setting (section 4; Table 1 at
r = 0): the distributed filter with K = 4 groups of N/K particles tracks as
well as the standard filter with N particles, and both beat the standard
filter with only N/K particles.  60 paired Monte Carlo runs (the same tracks
for the three methods), run as GPU batches."""
import pytest

from paper_1503_03769_amd.paper_table import run_config

pytestmark = pytest.mark.gpu


def test_distributed_filter_matches_full_filter(gpu):
    res = {m: run_config(m, 0.0, 60, 50)["mean_ospa"] for m in ("PHD", "DCPPHD", "partPHD")}
    print(res, flush=True)
    assert abs(res["DCPPHD"] - res["PHD"]) < 0.05 * res["PHD"], res
    assert res["partPHD"] > res["DCPPHD"] and res["partPHD"] > res["PHD"], res
