"""What the trained network gains over the method without it.

The committed weights (paper_2402_12833_amd/weights) were trained on the GPU
by the library's own kernels on fresh kappa fields (seeds 10000 + j).  On
held-out fields (seeds 900000 + i) of the same distribution the solve with
the learned direction appended must converge to the same tolerance (true
FP64 residual) in fewer iterations than the plain solve.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2402_12833_amd as amg  # noqa: E402
from paper_2402_12833_amd import train  # noqa: E402
import workloads as W  # noqa: E402


@pytest.fixture(scope="module")
def net():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    amg.load()
    nw = amg.Network(127)
    train.load_weights(nw)
    yield nw
    nw.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_learned_direction_reduces_iterations(net, precision):
    rows = train.evaluate(net, [W.TEST_KAPPA_SEED0 + i for i in range(3)], precision=precision, repeats=1)
    for row in rows:
        p, l = row["plain"], row["learned"]
        print(f"seed {row['seed']} precision {precision}: plain {p['iterations']} its {p['ms']:.1f} ms, "
              f"learned {l['iterations']} its {l['ms']:.1f} ms")
        assert p["status"] == amg.OK and l["status"] == amg.OK
        assert l["true_relres"] <= 1e-8 * 1.01 and p["true_relres"] <= 1e-8 * 1.01
        assert l["iterations"] < p["iterations"]
    mean_p = np.mean([r["plain"]["iterations"] for r in rows])
    mean_l = np.mean([r["learned"]["iterations"] for r in rows])
    assert mean_l <= 0.95 * mean_p
