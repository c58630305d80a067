"""What the learned cost model gains (GPU: the MLP trains on libparaiso's own kernels).

Replays the exhaustive benchmark database of the 512^3 FP32 box (every variant
measured on an MI355X) and runs MLP-guided, random and PAGSA search with the
same budget, over 15 seeds each: 10% of the exhaustive benchmark time (the
MLP's pick within 5% of the optimum), and 5%, where the search without the
model no longer finds the optimum on every seed.
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
    # the MLP pick is within 5% of the exhaustive optimum (median over seeds, and every seed)
    assert out["mlp_median"] >= 0.95 and out["mlp_min"] >= 0.95
    # and the model beats the searches without it at the same budget
    assert out["mlp_median"] >= out["random_median"] and out["mlp_median"] >= out["pagsa_median"]
    assert out["mlp_anytime_median"] > out["random_anytime_median"]
    assert out["mlp_anytime_median"] > out["pagsa_anytime_median"]


def test_mlp_gain_on_box512_at_5_percent():
    db = DB(os.path.join(DATA, "box512_f32.jsonl"))
    out = cli.gain_study(db, 3, 4, seeds=15, frac=0.05, log=print)
    print({k: v for k, v in out.items() if k != "runs"})
    assert out["budget"] <= 0.05 * out["exhaustive_cost"] + 1e-9
    assert out["mlp_median"] >= 0.95
    # best found: the model finds the optimum on more seeds than PAGSA and random,
    # and its mean and worst best-found fractions are higher
    assert out["mlp_hits"] > out["pagsa_hits"] and out["mlp_hits"] > out["random_hits"]
    assert out["mlp_mean"] > out["pagsa_mean"] and out["mlp_mean"] > out["random_mean"]
    assert out["mlp_min"] > out["pagsa_min"] and out["mlp_min"] > out["random_min"]
    assert out["mlp_anytime_median"] > out["pagsa_anytime_median"]
