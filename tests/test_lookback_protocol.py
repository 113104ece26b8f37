"""A host model of the single-pass integral histogram's carry protocol (decoupled look-back
between tiles), run under randomised wave schedules.

Each tile is a coroutine that follows the kernel's steps: publish the row and column totals
as aggregate records; look back up the tile column and along the tile row, a window of tiles
per poll, adding aggregates until an inclusive record; publish the inclusive records; publish
the total column carry and look back along the tile row for the corner carry (the nearest
inclusive record of the window ends it); then form every entry of its part of the 2-D
prefix (Eq. 8 for one plane).  A poll that finds a wanted record absent yields, and the
scheduler runs another wave.  Tickets go out in row-major order, a bounded number of waves
is resident, and a new wave starts only when a slot frees, so a wave waits only on waves
that already run.

The model must finish under every schedule (no wave waits forever) and give the exact 2-D
prefix sums, which numpy's cumulative sums fix independently.  The kernel's integer results
do not depend on the order the records arrive in; this checks that the protocol guarantees
it."""
import numpy as np
import pytest

AGG, INCL = 1, 2


class Records:
    """Record words: absent (None) or (state, count)."""

    def __init__(self):
        self.words = {}

    def put(self, key, state, count):
        self.words[key] = (state, count)

    def get(self, key):
        return self.words.get(key)


def look_back(rec, keys_of, n_back, window, slots):
    """Generator: sums, per slot, the counts of the records of the 1st, 2nd, ... tile back
    until a slot meets an inclusive record; polls `window` tiles at a time and yields while a
    wanted record of the window is absent.  Returns the per-slot sums."""
    acc = [0] * slots
    done = [n_back == 0] * slots
    base = 0
    while base < n_back and not all(done):
        jn = min(window, n_back - base)
        while True:
            words = [[rec.get(keys_of(base + j, s)) if not done[s] else (INCL, 0)
                      for s in range(slots)] for j in range(jn)]
            if all(w is not None for row in words for w in row):
                break
            yield
        for j in range(jn):
            for s in range(slots):
                if not done[s]:
                    state, count = words[j][s]
                    acc[s] += count
                    done[s] = state == INCL
        base += jn
    return acc


def corner_look_back(rec, key_of, n_back, window):
    """Generator: the corner carry's look-back (one plane): the records of up to `window` tiles
    are requested together; the nearest inclusive one ends the sum, which holds every count
    up to and including it."""
    total, done, base = 0, n_back == 0, 0
    while base < n_back and not done:
        jn = min(window, n_back - base)
        while True:
            words = [rec.get(key_of(base + j)) for j in range(jn)]
            if all(w is not None for w in words):
                break
            yield
        for state, count in words:
            total += count
            if state == INCL:
                done = True
                break
        base += jn
    return total


def tile_wave(t, img, th, tw, tiles_x, rec, out, windows):
    jc, jr, jk = windows
    H, W = img.shape
    tx, ty = t % tiles_x, t // tiles_x
    y0, x0 = ty * th, tx * tw
    blk = img[y0:y0 + th, x0:x0 + tw]
    rows, cols = blk.shape
    rt = blk.sum(axis=1)            # row totals
    cc = blk.sum(axis=0)            # column totals
    for r in range(rows):
        rec.put(("row", t, r), AGG, int(rt[r]))
    for c in range(cols):
        rec.put(("col", t, c), AGG, int(cc[c]))
    yield
    # column carries: up the tile column
    cse = yield from look_back(rec, lambda j, c: ("col", (ty - 1 - j) * tiles_x + tx, c),
                               ty, jc, cols)
    for c in range(cols):
        rec.put(("col", t, c), INCL, cse[c] + int(cc[c]))
    yield
    # row carries: along the tile row
    xc = yield from look_back(rec, lambda j, r: ("row", ty * tiles_x + tx - 1 - j, r),
                              tx, jr, rows)
    for r in range(rows):
        rec.put(("row", t, r), INCL, xc[r] + int(rt[r]))
    yield
    # corner: the tile's total column carry, then a look-back along the tile row
    ct = sum(cse)
    rec.put(("corner", t), AGG, ct)
    yield
    k = yield from corner_look_back(rec, lambda j: ("corner", ty * tiles_x + tx - 1 - j),
                                    tx, jk)
    rec.put(("corner", t), INCL, k + ct)
    # entries: own 2-D prefix + row carries summed down + column carries summed across + corner
    own = blk.cumsum(0).cumsum(1)
    down = np.cumsum(xc)[:, None]
    across = np.cumsum(cse)[None, :]
    out[y0:y0 + rows, x0:x0 + cols] = own + down + across + k


def run(img, th, tw, windows, resident, seed):
    H, W = img.shape
    tiles_x, tiles_y = -(-W // tw), -(-H // th)
    n = tiles_x * tiles_y
    rng = np.random.default_rng(seed)
    rec, out = Records(), np.full((H, W), -1, dtype=np.int64)
    running, ticket, steps = {}, 0, 0
    while ticket < n or running:
        while ticket < n and len(running) < resident:   # a freed slot takes the next ticket
            running[ticket] = tile_wave(ticket, img, th, tw, tiles_x, rec, out, windows)
            ticket += 1
        t = list(running)[rng.integers(len(running))]
        try:
            next(running[t])
        except StopIteration:
            del running[t]
        steps += 1
        assert steps < 200000, "a wave waits forever"
    return out


@pytest.mark.parametrize("H,W,th,tw", [(1, 1, 2, 4), (7, 9, 2, 4), (13, 37, 3, 4), (32, 16, 4, 4),
                                       (23, 41, 5, 8)])
@pytest.mark.parametrize("windows", [(1, 1, 1), (2, 2, 16), (4, 8, 8)])
@pytest.mark.parametrize("resident", [1, 3, 1000])
def test_look_back_protocol_gives_the_exact_prefix_under_any_schedule(H, W, th, tw, windows,
                                                                      resident):
    for seed in range(6):
        rng = np.random.default_rng(1000 * seed + H * W)
        img = (rng.random((H, W)) < 0.4).astype(np.int64)   # one plane's indicators
        got = run(img, th, tw, windows, resident, seed)
        assert np.array_equal(got, img.cumsum(0).cumsum(1))


def test_a_corner_look_back_that_skipped_the_nearest_inclusive_record_is_caught():
    """The model is sensitive: adding the counts past the first inclusive record (a plausible
    protocol slip) double-counts and the comparison fails."""
    def sloppy(rec, key_of, n_back, window):
        total = 0
        for j in range(n_back):
            while rec.get(key_of(j)) is None:
                yield
            total += rec.get(key_of(j))[1]
        return total
    img = np.ones((6, 12), dtype=np.int64)
    global corner_look_back
    saved = corner_look_back
    corner_look_back = sloppy
    try:
        got = run(img, 2, 4, (1, 1, 1), 1, 0)
    finally:
        corner_look_back = saved
    assert not np.array_equal(got, img.cumsum(0).cumsum(1))
