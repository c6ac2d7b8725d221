"""Host logic of the batch domain-size tuner (no GPU)."""
from paper_1104_3516_amd import tune


def test_domains_for_scales_with_contacts():
    assert tune.domains_for(100, 300) == 1
    assert tune.domains_for(262144, 150) == 2010
    assert tune.domains_for(65536, 300) == 251
    assert all(tune.domains_for(n, t) >= 1 for n in (1, 7, 300) for t in tune.CANDIDATES)


def test_cache_key_buckets():
    a = tune._key(2, 512, 5_580_310, "gpu")
    assert a == tune._key(2, 600, 5_000_000, "gpu")      # same buckets
    assert a != tune._key(3, 512, 5_580_310, "gpu")
    assert a != tune._key(2, 512, 5_580_310, "other")
