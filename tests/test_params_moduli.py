"""The library's parameter set-up (host code, no device): its moduli and NTT
roots equal the oracle's for every workload chain, and each root has order
exactly 2N (pinned on its own: psi^N = -1)."""
import pytest

from paper_2305_17341_amd import inputs as I


@pytest.mark.parametrize("chain", [I.TOY, I.TOY2, I.SMALL, I.MID, I.SERVE15, I.LARGE], ids=lambda c: c.name)
def test_moduli_and_roots_equal_the_oracles(oracle_mod, chain):
    from paper_2305_17341_amd import he
    mods, psi = he.params_moduli(chain.log_n, chain.q_bits, chain.p_bits)
    o = oracle_mod.Oracle(chain.log_n, chain.q_bits, chain.p_bits)
    assert mods == o.moduli
    assert psi == [o.psi(m) for m in range(len(mods))]
    N = chain.N
    for q, w in zip(mods, psi):
        assert q % (2 * N) == 1
        assert pow(w, N, q) == q - 1
