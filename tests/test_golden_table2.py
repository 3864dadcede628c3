"""The only numbers the paper prints for LP-SIFT itself are the feature-point
and match counts of Table 2 (Sec. 3), measured on images that are not
available. They bound the detector from above: every window of every L gives
at most one maximum and one minimum (Sec. 2.2, Eq. 2), so an image of H x W
has at most 2 sum_L ceil(H / L) ceil(W / L) feature points (the oracle's slot
count, partial windows at the right and bottom borders included), and the
paper's counts, which drop some candidates by a rule it does not state, must
lie below it; matched pairs (Sec. 2.4) cannot exceed the points of either
image."""
import os

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table2_lpsift.txt")


def rows():
    out = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, w, h, l1, l2, pa, pb, m = line.split()
        out.append((name, int(w), int(h), [int(l1), int(l2)], int(pa), int(pb), int(m)))
    return out


def test_table2_fixture_is_complete():
    names = [r[0] for r in rows()]
    assert names == ["mountain", "street_view", "terrain", "building", "campus_translation",
                     "campus_rotation"]


def test_printed_counts_lie_below_the_slot_count():
    for name, w, h, Ls, pa, pb, m in rows():
        slots = oracle.num_keypoints(h, w, Ls)
        by_hand = 2 * sum(-(-h // L) * -(-w // L) for L in Ls)
        assert slots == by_hand, name
        assert max(pa, pb) <= slots, name
        assert m <= min(pa, pb), name
