"""The pseudo-inverse entry point that allocates no device memory
(amgmpcg_gram_pinv_noalloc, for callers that cannot call hipMalloc) against
the allocating one (amgmpcg_gram_pinv), through the C ABI: two calls in a
row on the same GPU, the second with a smaller Gram, bit for bit, plus the
size limit of its static staging."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2402_12833_amd as amg  # noqa: E402
from oracle import mpcg  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    amg.load()


def gram(nb, seed, dup=False):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((50, nb)) * np.exp(rng.uniform(-3, 3, nb))
    if dup:
        B[:, -1] = 3.0 * B[:, 0]
    return B.T @ B


@pytest.mark.parametrize("sizes", [(7, 4), (8, 1), (6, 6)])
def test_noalloc_matches_allocating_entry_point(sizes):
    for i, nb in enumerate(sizes):
        for dup in (False, True):
            if dup and nb < 2:
                continue
            G = gram(nb, 10 * nb + i, dup)
            tau = mpcg.default_tau(nb)
            Gp_ref, rank_ref = amg.gram_pinv(G, tau)
            Gp, rank = amg.gram_pinv_noalloc(G, tau)
            assert rank == rank_ref, (nb, dup)
            assert np.array_equal(Gp, Gp_ref), (nb, dup)
            # and the result is the oracle's pseudo-inverse (the parity bar of
            # the allocating entry point)
            ref = mpcg.pinv_gram(G, tau)
            assert rank == ref.rank
            if not dup:
                np.testing.assert_allclose(Gp, ref.Gplus, rtol=1e-9, atol=1e-12 * np.abs(ref.Gplus).max())


def test_noalloc_rejects_sizes_beyond_the_staging():
    G = gram(9, 3)
    with pytest.raises(amg.AmgMpcgError) as e:
        amg.gram_pinv_noalloc(G, 1e-12)
    assert e.value.code == amg.INVALID_ARG
    # the next call still works
    Gp, rank = amg.gram_pinv_noalloc(gram(3, 4), 1e-12)
    assert rank == 3
