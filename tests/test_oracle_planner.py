"""Direct pins of the oracle's own level/scale rule (tower reuse, Section
4.3) against the paper: the level table of Section 4.4 (ResNet-20 20,
ResNet-18 18, ResNet-32 32 levels with every optimisation), the law that
tower reuse needs ceil(L / 2) of the levels a chain of primes ~ Delta needs,
and the worked example of Section 4.3.  OracleNetwork.schedule() applies the
same helper functions run() applies (the last test checks run() against it),
and nothing here imports the product's planner."""
import math

import numpy as np
import pytest

from oracle.ckks import Oracle
from oracle.network import OracleNetwork
from workloads import gen, nets
from workloads.params import balanced_chain, nearest_prime, resnet20_tower, small_tower

D = 2.0 ** 30


class _Chain:
    """The oracle's planner reads only the chain (q, L); a full context at
    N = 2^16 is not needed to plan."""

    def __init__(self, q):
        self.q = [int(x) for x in q]
        self.L = len(self.q) - 1


def _schedule(spec, q, delta=D):
    return OracleNetwork(_Chain(q), spec, delta, delta, delta).schedule()


def _levels_used(spec, q):
    sch = _schedule(spec, q)
    return len(q) - 1 - sch[-1]["level_out"], sum(s["rescale"] for s in sch)


def _lam(s):
    return int(round(math.log2(s) / 30))


def test_oracle_level_count_resnet20():
    """Section 4.4: ResNet-20 needs 20 levels, one rescale per level."""
    spec = nets.resnet_spec(seed=0, members=1, widths=(16, 32, 64), blocks=3, classes=10, image=(3, 32, 32), k=4,
                            calib=1)
    assert _levels_used(spec, resnet20_tower().q) == (20, 20)


@pytest.mark.parametrize("widths,blocks,levels", [((64, 128, 256, 512), 2, 18), ((16, 32, 64), 5, 32)])
def test_oracle_level_counts_resnet18_resnet32(widths, blocks, levels):
    spec = nets.resnet_spec(seed=0, members=1, widths=widths, blocks=blocks, classes=10, image=(3, 32, 32), k=4,
                            calib=1)
    used, _ = _levels_used(spec, resnet20_tower(levels=levels + 2).q)
    assert used == levels


def test_oracle_tower_reuse_halves_the_levels():
    """39 levels on a chain of primes ~ Delta (every multiplicative layer
    rescales), 20 = ceil(39 / 2) with q_i ~ Delta^2."""
    spec = nets.resnet_spec(seed=0, members=1, widths=(16, 32, 64), blocks=3, classes=10, image=(3, 32, 32), k=4,
                            calib=1)
    two_n = 2 << 16
    q = balanced_chain([30] * 48, two_n)
    q = [nearest_prime(40, two_n, exclude=q)] + q
    std, rescales = _levels_used(spec, q)
    tower, _ = _levels_used(spec, resnet20_tower().q)
    assert std == 39 and rescales == 39
    assert tower == 20 == -(-std // 2)


def test_oracle_tower_reuse_worked_example():
    """Section 4.3: at q_i ~ Delta^2 an activation of an input at sublevel 1
    stays at sublevel 2 (no rescale); the next convolution (weights at
    sublevel 1) reaches 3 > 2 and rescales back to sublevel 1."""
    spec = nets.vgg_spec(seed=1, widths=(4, 4), pool_after=(), classes=2, image=(3, 8, 8), k=4, calib=1)
    q = resnet20_tower(levels=4).q
    conv0, act0, conv1 = _schedule(spec, q)[:3]
    assert _lam(float(q[conv1["level_in"]])) == 2
    assert _lam(act0["scale_in"]) == 1 and not act0["rescale"] and _lam(act0["scale_out"]) == 2
    assert _lam(conv1["scale_in"]) == 2
    assert _lam(conv1["scale_out"] / conv1["scale_in"]) == 1
    assert _lam(conv1["scale_out"]) == 3 and conv1["rescale"]
    assert _lam(conv1["scale_out_final"]) == 1


def test_oracle_standard_chain_rescales_after_every_product():
    """With every prime ~ Delta the rule rescales after every multiplicative
    layer (the standard chain)."""
    from workloads.params import tiny
    ps = tiny()
    spec = nets.tiny_spec(0)
    sch = OracleNetwork(_Chain(ps.q), spec, 2.0 ** 40, 2.0 ** 34, 2.0 ** 40).schedule()
    assert [s["rescale"] for s in sch] == [True, True] and sch[-1]["level_out"] == 0


def test_oracle_run_follows_its_schedule():
    """Every output ciphertext of run() has the level and scale schedule()
    gives for its layer."""
    ps = small_tower(logN=12, levels=4)
    o = Oracle.from_params(ps)
    spec = nets.vgg_spec(seed=2, widths=(4, 4), pool_after=(0,), classes=3, image=(3, 8, 8), k=4, calib=2)
    net = OracleNetwork(o, spec, D, D, D)
    sk = o.secret_key(3)
    rlk = o.relin_key(sk)
    gk = {o.galois_elt(s): o.galois_key(sk, o.galois_elt(s)) for s in net.steps()}
    seen = []
    net.run(sk, net.encrypt_image(sk, gen.images(2, 1, 3, 8, 8)[0], 10), rlk, gk,
            hook=lambda ly, outs: seen.append((ly["name"], outs[0].level, outs[0].scale)))
    sch = net.schedule()
    assert [n for n, _, _ in seen] == [s["name"] for s in sch]
    for (n, lv, sc), s in zip(seen, sch):
        assert lv == s["level_out"] and sc == s["scale_out_final"], n
