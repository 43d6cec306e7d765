"""Pins for the oracle's channel table against Eq. C_quark and Eq. C_gluon.

The paper prints, for each species, which 2->2 processes enter its collision
term and with which coefficient (1/2 for identical initial particles).  The
oracle's per-channel coefficient sigma must reproduce every printed term, and
the symmetric-sampling weights w must sum, over the channels of one reaction,
to the same coefficients (which is what makes the symmetric estimator unbiased).
"""
from collections import Counter, defaultdict

import pytest

U, D, S, UB, DB, SB, G = range(7)
Q, QB = (U, D, S), (UB, DB, SB)


def rkey(a, b, c, d):
    """A reaction {a,b} <-> {c,d}, direction-free."""
    return frozenset([tuple(sorted((a, b))), tuple(sorted((c, d)))])


def paper_coefficients():
    """(reaction, species) -> coefficient, read off Eq. C_quark / Eq. C_gluon."""
    coef = {}
    for i in range(3):
        qa, qab = Q[i], QB[i]
        for x, xb in ((qa, qab), (qab, qa)):          # quark and, by C, antiquark
            coef[(rkey(x, x, x, x), x)] = 0.5         # 1/2 C_{qa qa <-> qa qa}
            coef[(rkey(x, xb, x, xb), x)] = 1.0       # C_{qa qbar_a <-> qa qbar_a}
            coef[(rkey(G, G, x, xb), x)] = 0.5        # 1/2 C_{gg <-> qa qbar_a}
            coef[(rkey(x, G, x, G), x)] = 1.0         # C_{qa g <-> qa g}
            for j in range(3):
                if j == i:
                    continue
                y, yb = (Q[j], QB[j]) if x in Q else (QB[j], Q[j])
                coef[(rkey(x, y, x, y), x)] = 1.0     # C_{qa qb}
                coef[(rkey(x, yb, x, yb), x)] = 1.0   # C_{qa qbar_b}
                coef[(rkey(y, yb, x, xb), x)] = 1.0   # C_{qb qbar_b <-> qa qbar_a}
        # gluon: sum_a (C_{g qa} + C_{g qbar_a} + C_{qa qbar_a <-> gg})
        coef[(rkey(G, qa, G, qa), G)] = 1.0
        coef[(rkey(G, qab, G, qab), G)] = 1.0
        coef[(rkey(qa, qab, G, G), G)] = 1.0
    coef[(rkey(G, G, G, G), G)] = 0.5                 # 1/2 C_{gg <-> gg}
    return coef


def test_counts(O):
    ch = O.channels(O.Grid(species_mask=0x7F))
    assert len(ch) == 70
    assert Counter(c["sp"][0] for c in ch) == {sp: 10 for sp in range(7)}
    assert len({rkey(*c["sp"]) for c in ch}) == 34
    assert len({c["code"] for c in ch}) == 70
    assert Counter(c["row"] for c in ch) == {1: 24, 2: 6, 3: 6, 4: 12, 5: 9, 6: 12, 7: 1}


def test_sigma_reproduces_paper_coefficients(O):
    ch = O.channels(O.Grid(species_mask=0x7F))
    expected = paper_coefficients()
    got = {(rkey(*c["sp"]), c["sp"][0]): c["sigma"] for c in ch}
    assert set(got) == set(expected)
    for k, v in expected.items():
        assert got[k] == pytest.approx(v, abs=0, rel=1e-15), k


def test_symmetric_weights_are_unbiased(O):
    """Sum over a reaction's channels of w * n_Y must equal the paper's coefficient
    for every species Y of the reaction (expected symmetric deposit = sigma C)."""
    ch = O.channels(O.Grid(species_mask=0x7F))
    expected = paper_coefficients()
    by_reaction = defaultdict(list)
    for c in ch:
        by_reaction[rkey(*c["sp"])].append(c)
    for key, chans in by_reaction.items():
        tup = chans[0]["sp"]
        for Y in set(tup):
            nY = sum(1 for x in tup if x == Y)
            total = sum(c["w"] * nY for c in chans)
            assert total == pytest.approx(expected[(key, Y)], rel=1e-15)


def test_channel_order_keeps_t_channel_partner(O):
    """Rows whose |M|^2 is not t<->u symmetric: position 3 must be the t-channel
    partner of position 1 (same line through the exchanged gluon)."""
    for c in O.channels(O.Grid(species_mask=0x7F)):
        sp = c["sp"]
        if c["row"] in (1, 3, 6):
            assert sp[2] == sp[0] and sp[3] == sp[1], c
        if c["row"] == 4:
            assert (sp[0] in Q) == (sp[2] in Q), c


def test_masks_select_reactions(O):
    assert [c["row"] for c in O.channels(O.Grid(species_mask=1 << G))] == [7]
    assert O.channels(O.Grid(species_mask=0x7F, row_mask=0)) == []
    only_u = O.channels(O.Grid(species_mask=1 << U))
    assert [c["sp"] for c in only_u] == [(U, U, U, U)]
    assert len(O.channels(O.Grid(species_mask=0x7F, row_mask=1 << 6))) == 1
