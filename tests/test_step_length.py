"""The host tabulates the comoving step length of a level-l leaf as
(box / n0) / 2^l / N (N steps per leaf cell, Sect. 2.2), and the kernels
compute it as ldexp((box / n0) / N, -l) instead of reading the table with a
per-lane index.  The two agree bit for bit because scaling by a power of two
is exact and commutes with rounding; this checks it over the box sizes,
coarse counts, levels and step counts the library accepts."""
import math

import numpy as np


def test_step_length_is_exact_power_of_two_scaling():
    rng = np.random.default_rng(11)
    n = 0
    for box in np.concatenate([rng.uniform(1.0, 1.0e4, 400), [500.0, 2000.0, 1.0, 1.0e4]]):
        for n0 in (1, 2, 4, 64, 128, 512, 1024):
            for N in (1, 2, 3, 4, 5, 7, 10, 16, 33, 64):
                h0 = float(box) / n0
                ds0 = h0 / N
                for level in range(0, 11):
                    table = h0 / float(1 << level) / N
                    assert table == math.ldexp(ds0, -level), (box, n0, N, level)
                    n += 1
    assert n > 300000
