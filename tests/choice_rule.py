"""The library's built-in configuration rule (csrc/mgemm_api.hip) written out in
Python, without split-k, so tests can score it on the tuner database: the
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


def library_choice(tables, dt, m, n, k):
    c = pref_choice(dt, m, n)
    whole = not gen.three_stage_ineligible(dt, n, k)
    if not whole or c[5] != 2:
        c = tables[int(whole)][dt].get(gen.cell_of(m, n, k), c)
    return c
