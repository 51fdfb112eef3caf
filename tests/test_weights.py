"""The shipped opening-parameter network (paper_1112_4539_amd/weights/theta_clumpy4m.json): a
well-formed file of the network the library's MLP kernels run (Sec. 4.4, theta as the opening
parameter of Eq. (2)), checked on the CPU without loading the library."""
import json
import math
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_1112_4539_amd", "weights", "theta_clumpy4m.json")


def test_shipped_weights_well_formed():
    rec = json.load(open(WEIGHTS))
    assert rec["format"] == "theta-mlp-8-64-64-1"
    # W1 [64x8], b1 [64], W2 [64x64], b2 [64], w3 [64], b3 [1]
    assert rec["n_param"] == len(rec["params"]) == 8 * 64 + 64 + 64 * 64 + 64 + 64 + 1
    assert all(math.isfinite(x) for x in rec["params"])
    # norm: 8 feature means, then 8 inverse standard deviations
    assert len(rec["norm"]) == 16 and all(math.isfinite(x) for x in rec["norm"])
    assert all(x > 0 for x in rec["norm"][8:])
    # every value is an FP32 number (the file holds the FP32 parameters exactly)
    import numpy as np
    p = np.asarray(rec["params"], np.float64)
    assert np.array_equal(p.astype(np.float32).astype(np.float64), p)
    info = rec["info"]
    assert "seeds 300-331" in info["fields"] and info["label_target_rms"] == 1e-3
    assert info["sampled_groups_per_field"] == 4096 and info["rows"] == 32 * 4096
    assert info["loss_first_last"][1] < info["loss_first_last"][0]
