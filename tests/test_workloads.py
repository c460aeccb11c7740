"""The seeded input generators: deterministic, and batches drawn as stated
(sizes from the given set independently per axis, one bed seed per
instance, inflow discharge in the given range)."""
import numpy as np

from paper_1608_06721_amd import workloads as W


def test_batch_channels_is_deterministic_and_as_stated():
    a = W.batch_channels(16, n_levels=5)
    b = W.batch_channels(16, n_levels=5)
    for p, q in zip(a, b):
        assert p.name == q.name
        np.testing.assert_array_equal(p.z, q.z)
        np.testing.assert_array_equal(p.U0, q.U0)
    assert {p.nx for p in a} <= {128, 256, 384, 512}
    assert {p.ny for p in a} <= {128, 256, 384, 512}
    assert len({(p.nx, p.ny) for p in a}) > 4
    qs = [p.bc[0][2] for p in a]
    assert all(0.5 <= q <= 2.0 for q in qs) and len(set(qs)) == len(qs)
    for p in a:
        assert p.params["n_levels"] == 5
        assert p.z.shape == (p.ny, p.nx) and p.U0.shape == (3, p.ny, p.nx)
        assert p.nx % 32 == 0 and p.ny % 32 == 0
    # different instances have different beds
    assert not np.array_equal(a[0].z[:64, :64], a[1].z[:64, :64])
