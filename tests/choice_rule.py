"""The library's built-in configuration rule (csrc/mgemm_api.hip) written out in
Python, without a loaded model.

library_choice (no k cut, for scoring the rule on the tuner database): for rows
that are whole 16-byte loads, the three-stage tile that fills the compute units'
rounds best if one fills them well enough; otherwise the preference list, replaced
by the cell's measured configuration for rows that are not whole 16-byte loads, or
where the list names a two-stage configuration.

library_plan (what mgemm_choice reports): first split-k, for k >= 2048 or a shape
outside the measured range, where the preferred tile is a small one that leaves the
compute units short of work; then, for rows of whole 16-byte loads, a split tail
where its time estimate beats the best single three-stage tile by 5 % (2 % where
that tile is 128 x 128 or 256 x 128); then library_choice."""
from paper_1706_10086_amd.csrc import gen_choice_table as gen

# the preference list: (configuration, minimum C tiles to take it)
PREF = {0: [((256, 128, 16, 8, 2, 2, 2), 512), ((128, 128, 16, 8, 2, 2, 2), 256),
            ((128, 64, 32, 4, 4, 0, 2), 256), ((64, 64, 16, 4, 2, 1, 0), 256),
            ((32, 32, 16, 1, 2, 1, 0), 0)],
        1: [((256, 128, 32, 8, 4, 2, 2), 512), ((128, 128, 32, 8, 4, 2, 2), 256),
            ((128, 64, 32, 4, 4, 1, 0), 256), ((64, 64, 16, 4, 2, 1, 0), 256),
            ((32, 32, 16, 1, 2, 1, 0), 0)]}


def pref_choice(dt, m, n):
    pl = PREF[dt]
    for i, (c, min_tiles) in enumerate(pl):
        if i + 1 < len(pl) and (-(-m // c[0])) * (-(-n // c[1])) < min_tiles:
            continue
        return c


# three-stage tiles and the rates (TFLOP/s) the library's wave-fill rule weighs them
# by, and the compute units of an MI355X
PIPE_RATES = {0: [((256, 128, 16, 8, 2, 2, 2), 72.5), ((128, 128, 16, 8, 2, 2, 2), 70.4),
                  ((64, 64, 32, 4, 2, 2, 1), 54.2)],
              1: [((256, 128, 32, 8, 4, 2, 2), 141.0), ((128, 128, 32, 8, 4, 2, 2), 135.1),
                  ((64, 64, 32, 4, 4, 2, 1), 120.6)]}
CUS = 256
WAVE_FILL_MIN = 0.8


def _best_filled_pipe(dt, m, n):
    """(tile, rate x fill, fill) of the three-stage tile with the highest rate x
    fill of its rounds of CUS work-groups."""
    best, score, fill_best = None, 0.0, 0.0
    for c, rate in PIPE_RATES[dt]:
        t = (-(-m // c[0])) * (-(-n // c[1]))
        fill = t / (-(-t // CUS) * CUS)
        if rate * fill > score:
            best, score, fill_best = c, rate * fill, fill
    return best, score, fill_best


def wave_filled_pipe(dt, m, n):
    """The three-stage tile with the highest rate x fill of its rounds of CUS
    work-groups, if that fill is at least WAVE_FILL_MIN; else None."""
    best, _, fill_best = _best_filled_pipe(dt, m, n)
    return best if fill_best >= WAVE_FILL_MIN else None


def library_choice(tables, dt, m, n, k):
    c = pref_choice(dt, m, n)
    whole = not gen.three_stage_ineligible(dt, n, k)
    if whole:
        q = wave_filled_pipe(dt, m, n)
        if q is not None:
            return q
    if not whole or c[5] != 2:
        c = tables[int(whole)][dt].get(gen.cell_of(m, n, k), c)
    return c


# split-k: k ranges are multiples of 256, at most 16 of them; the built-in choice
# cuts k first from k = 2048 and outside the measured range [64, 16384]
SPLITK_MIN_K, SPLITK_FIRST_K, SPLITK_MAX = 256, 2048, 16
MEASURED_LO, MEASURED_HI = 64, 16384
# the two-stage tiles registered with a split-k kernel, and the three-stage
# 128 x 128 tile that runs the three-stage split-k and the split tail
TWO_STAGE_SPLITK = {0: {(64, 64, 16, 4, 2, 1, 0), (32, 32, 16, 1, 2, 1, 0)}, 1: set()}
PIPE128 = {0: PIPE_RATES[0][1][0], 1: PIPE_RATES[1][1][0]}
# the split tail's estimate: the tail at this fraction of the tile's rate, the sum
# of the partial planes at this many bytes per second, and the gain it must reach
# over the best single tile (over a 128 x 128 or 256 x 128 one: TAIL_GAIN_LARGE)
TAIL_RATE_FACTOR, SUM_BYTES_PER_S, TAIL_GAIN, TAIL_GAIN_LARGE = 0.8, 4e12, 1.05, 1.02


def _cdiv(a, b):
    return -(-a // b)


def cut_k(k, want):
    """The number of k ranges for about ``want`` ranges of k (1: no cut)."""
    want = min(want, k // SPLITK_MIN_K, SPLITK_MAX)
    if want < 2:
        return 1
    kc = _cdiv(_cdiv(k, want), SPLITK_MIN_K) * SPLITK_MIN_K
    s = _cdiv(k, kc)
    return s if s >= 2 else 1


def rows16(dt, n, lda, ldb):
    """Whether the rows of A and B are whole 16-byte loads (16-byte bases)."""
    epu = 4 if dt == 1 else 2
    return n % epu == 0 and lda % epu == 0 and ldb % epu == 0


def pipe_split_eligible(dt, n, k, lda, ldb):
    """The three-stage 128 x 128 split-k's requirements: 16-byte rows and 32-bit
    panel offsets."""
    es = 4 if dt == 1 else 8
    bk = 32 if dt == 1 else 16
    return (k >= 1 and n >= 16 // es and rows16(dt, n, lda, ldb)
            and 128 * lda * es < 2 ** 31 and (bk * ldb + 128) * es < 2 ** 31)


def splitk_plan(dt, m, n, k, lda, ldb, pref):
    """(k ranges, configuration that runs them) for the preferred tile ``pref``:
    only a 64 x 64 or smaller tile that leaves fewer than about four work-groups
    per compute unit is cut; the three-stage 128 x 128 tile takes the ranges where
    its S x tiles fill at least 3/4 of the compute units, else the two-stage tile
    its own (FP64 only)."""
    tiles = _cdiv(m, pref[0]) * _cdiv(n, pref[1])
    if pref[0] * pref[1] > 64 * 64:
        return 1, None
    want = _cdiv(4 * CUS, tiles)
    if want < 2:
        return 1, None
    if pipe_split_eligible(dt, n, k, lda, ldb):
        t128 = _cdiv(m, 128) * _cdiv(n, 128)
        s = cut_k(k, CUS // t128)
        if s > 1 and 4 * t128 * s >= 3 * CUS:
            return s, PIPE128[dt]
    if pref not in TWO_STAGE_SPLITK[dt]:
        return 1, None
    s = cut_k(k, want)
    return (s, pref) if s > 1 else (1, None)


def split_tail(dt, m, n, k, lda, ldb, plain_tf, plain_large=False):
    """(k ranges, rows run whole) of a split tail with the 128 x 128 tile, or None:
    the tile rows that fill whole rounds run whole, the other rows with k cut so
    that S x their tiles fit the compute units; taken when the estimate beats
    plain_tf (the best single tile's rate x fill) by TAIL_GAIN, or by
    TAIL_GAIN_LARGE where that tile is 128 x 128 or larger (plain_large)."""
    if not pipe_split_eligible(dt, n, k, lda, ldb):
        return None
    rate = PIPE_RATES[dt][1][1]
    tm, tn = _cdiv(m, 128), _cdiv(n, 128)
    full = tm * tn // CUS
    if full < 1:
        return None
    r1 = full * CUS // tn
    if r1 < 1 or r1 >= tm:
        return None
    t1, t2 = r1 * tn, (tm - r1) * tn
    s = cut_k(k, CUS // t2)
    if s < 2:
        return None
    main_rows = r1 * 128
    w = 2.0 * m * n * k * 1e-12
    wm = w * main_rows / m
    fill_m = t1 / (_cdiv(t1, CUS) * CUS)
    fill_t = min(1.0, t2 * s / CUS)
    es = 4 if dt == 1 else 8
    t = (wm / (rate * fill_m) + (w - wm) / (rate * TAIL_RATE_FACTOR * fill_t)
         + (s + 2) * (m - main_rows) * n * es / SUM_BYTES_PER_S)
    if w / t < (TAIL_GAIN_LARGE if plain_large else TAIL_GAIN) * plain_tf:
        return None
    return s, main_rows


def library_plan(tables, dt, m, n, k, lda=None, ldb=None):
    """(configuration, k ranges, rows run whole) as mgemm_choice reports them for
    an m x n x k product with 16-byte aligned bases: rows run whole are m with no
    cut, 0 for a plain split-k and the rows before the tail for a split tail; the
    configuration of a three-stage split is the 128 x 128 tile."""
    lda = k if lda is None else lda
    ldb = n if ldb is None else ldb
    pref = pref_choice(dt, m, n)
    in_range = all(MEASURED_LO <= x <= MEASURED_HI for x in (m, n, k))
    if not in_range or k >= SPLITK_FIRST_K:
        s, c = splitk_plan(dt, m, n, k, lda, ldb, pref)
        if s > 1:
            return c, s, 0
    whole = rows16(dt, n, lda, ldb)
    if whole:
        q, score, fill = _best_filled_pipe(dt, m, n)
        tail = split_tail(dt, m, n, k, lda, ldb, score, q[0] * q[1] >= 128 * 128)
        if tail is not None:
            return PIPE128[dt], tail[0], tail[1]
        if fill >= WAVE_FILL_MIN:
            return q, 1, m
    c = pref
    if in_range and (not whole or c[5] != 2):
        c = tables[int(whole)][dt].get(gen.cell_of(m, n, k), c)
    return c, 1, m
