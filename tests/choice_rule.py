"""The library's built-in configuration rule (csrc/mgemm_api.hip) written out in
Python, without split-k and without a loaded model, so tests can score it on the
tuner database: for rows that are whole 16-byte loads, the three-stage tile that
fills the compute units' rounds best if one fills them well enough; otherwise the
preference list, replaced by the cell's measured configuration for rows that are
not whole 16-byte loads, or where the list names a two-stage configuration."""
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


def wave_filled_pipe(dt, m, n):
    """The three-stage tile with the highest rate x fill of its rounds of CUS
    work-groups, if that fill is at least WAVE_FILL_MIN; else None."""
    best, score, fill_best = None, 0.0, 0.0
    for c, rate in PIPE_RATES[dt]:
        t = (-(-m // c[0])) * (-(-n // c[1]))
        fill = t / (-(-t // CUS) * CUS)
        if rate * fill > score:
            best, score, fill_best = c, rate * fill, fill
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
