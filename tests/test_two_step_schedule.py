"""Host-side check of the iteration schedule the two-step kernels' 1/Sigma-hat
ring relies on (csrc/tk_kernels.hip, march2 and march2c).

Level 1 forms half row r and node row r-1 in iteration r and leaves each
point's 1/Sigma-hat in ring slot S (three slots, S the iteration's index
mod 3); level 2 forms half row r-3 and node row r-4 in iteration r and reads
slot S at the start of the iteration, before level 1 refills it.  The
reuse is exact only if, for every grid height and every chunk the work list
can make, each row level 2 forms is the row level 1 left in that slot: this
test replays the two marches' row conditions (the whole-strip bounds, and
the chunk bounds of chunk2_of with the work list's chunking rule) and checks
that.  The GPU tests check the kernels' results bitwise against the one-step
kernel; this pins the argument for grids and chunkings they do not run."""


def chunk_bounds(nt, j0, j1):
    north, south = j0 == 0, j1 == nt
    return dict(r_lo=1 if north else j0 - 3, h1_hi=nt - 2 if south else j1 + 2,
                v_lo=1 if north else j0 - 2, v_hi=nt - 2 if south else j1 + 1,
                g_lo=1 if north else j0 - 1, g_hi=nt - 2 if south else j1,
                o_lo=1 if north else j0, o_hi=nt - 2 if south else j1 - 1)


def replay(r_lo, r_hi, put_h, put_n, get_h, get_n):
    """Run iterations r_lo..r_hi; put_*/get_* say whether level 1 forms (and
    leaves) half row r / node row r-1 and level 2 forms half row r-3 / node
    row r-4 in iteration r.  Returns the number of reuses checked."""
    half, node = [None] * 3, [None] * 3
    n = 0
    for r in range(r_lo, r_hi + 1):
        s = (r - r_lo) % 3
        h_read, n_read = half[s], node[s]  # read at the start of the iteration
        if put_h(r):
            half[s] = r
        if put_n(r):
            node[s] = r - 1
        if get_h(r):
            assert h_read == r - 3, (r, h_read)
            n += 1
        if get_n(r):
            assert n_read == r - 4, (r, n_read)
            n += 1
    return n


def test_whole_strip_schedule():
    for nt in range(5, 300):
        n = replay(1, nt + 2,
                   put_h=lambda r: r <= nt - 2, put_n=lambda r: 2 <= r <= nt - 1,
                   get_h=lambda r: 4 <= r <= nt + 1, get_n=lambda r: 5 <= r <= nt + 2)
        # level 2 forms every interior half row and node row once
        assert n == 2 * (nt - 2)


def test_chunk_schedules():
    min_rows = 4  # the two-step kernels' smallest chunk
    for nt in range(5, 140):
        for rows in list(range(min_rows, 40)) + [nt]:
            covered_h, covered_n = [], []
            j0 = 0
            while j0 < nt:
                j1 = min(nt, j0 + rows)
                if 0 < nt - j1 < min_rows:
                    j1 = nt
                B = chunk_bounds(nt, j0, j1)
                r_hi = B["o_hi"] + 4
                replay(B["r_lo"], r_hi,
                       put_h=lambda r: r <= B["h1_hi"],
                       put_n=lambda r: B["v_lo"] <= r - 1 <= B["v_hi"],
                       get_h=lambda r: B["g_lo"] <= r - 3 <= B["g_hi"],
                       get_n=lambda r: B["o_lo"] <= r - 4 <= B["o_hi"])
                covered_h += range(B["g_lo"], B["g_hi"] + 1)
                covered_n += range(B["o_lo"], B["o_hi"] + 1)
                if j1 == nt:
                    break
                j0 = j1
            # the chunks write every interior node row exactly once
            assert sorted(covered_n) == list(range(1, nt - 1)), (nt, rows)
            assert set(covered_h) == set(range(1, nt - 1)), (nt, rows)


def test_a_wrong_schedule_is_caught():
    # a ring one slot too short for the three-row lag fails the check
    import pytest
    with pytest.raises(AssertionError):
        half, nt = [None] * 2, 20
        for r in range(1, nt + 3):
            s = (r - 1) % 2
            h_read = half[s]
            if r <= nt - 2:
                half[s] = r
            if 4 <= r <= nt + 1:
                assert h_read == r - 3
