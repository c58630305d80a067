"""What the learned cost model gains (GPU: the MLP trains on libparaiso's own kernels).

Replays the exhaustive benchmark database of the 512^3 FP32 box (every variant
measured on an MI355X) and runs MLP-guided, random and PAGSA search with the
same budget, 10% of the exhaustive benchmark time, over 15 seeds each.
"""
import os

import pytest

from paper_1204_4779_amd.tuner import __main__ as cli
from paper_1204_4779_amd.tuner.db import DB

pytestmark = pytest.mark.gpu

DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_1204_4779_amd", "tuner", "data")


def test_mlp_gain_on_box512():
    db = DB(os.path.join(DATA, "box512_f32.jsonl"))
    out = cli.gain_study(db, 3, 4, seeds=15, frac=0.1, log=print)
    print({k: v for k, v in out.items() if k != "runs"})
    assert out["budget"] <= 0.1 * out["exhaustive_cost"] + 1e-9
    # the MLP pick is within 5% of the exhaustive optimum (median over seeds)
    assert out["mlp_median"] >= 0.95
    # and the model beats the searches without it at the same budget
    assert out["mlp_median"] >= out["random_median"] and out["mlp_median"] >= out["pagsa_median"]
    assert out["mlp_anytime_median"] > out["random_anytime_median"]
    assert out["mlp_anytime_median"] > out["pagsa_anytime_median"]
