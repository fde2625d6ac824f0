"""The autotuner's host-side choice (no GPU): the fastest median wins unless
the library's built-in entry ties with it within the tolerance."""
from paper_1206_5878_amd import tune


def row(sorted_, blocks, chunk, ms):
    return dict(sorted=sorted_, bracket_blocks=blocks, trial_chunk=chunk, ms_per_step=ms)


def test_candidates_cover_both_forms():
    c = list(tune.candidates())
    assert {x["sorted"] for x in c} == {0, 1}
    assert all(x["trial_chunk"] % 64 == 0 and 64 <= x["trial_chunk"] <= 1024 for x in c)
    assert len({tuple(sorted(x.items())) for x in c}) == len(c)


def test_pick_keeps_a_tied_incumbent():
    rows = [row(0, 512, 128, 1.000), row(0, 1024, 128, 0.990), row(1, 1024, 128, 1.50)]
    inc = dict(min_cap=0, sorted=0, bracket_blocks=512, trial_chunk=128)
    assert tune.pick(rows, inc)["bracket_blocks"] == 512  # within TIE of the fastest


def test_pick_takes_a_clearly_faster_candidate():
    rows = [row(0, 512, 128, 1.10), row(0, 1024, 128, 1.00)]
    inc = dict(min_cap=0, sorted=0, bracket_blocks=512, trial_chunk=128)
    assert tune.pick(rows, inc)["bracket_blocks"] == 1024
    # an incumbent that is not among the candidates changes nothing
    inc = dict(min_cap=0, sorted=0, bracket_blocks=4096, trial_chunk=128)
    assert tune.pick(rows, inc)["bracket_blocks"] == 1024
