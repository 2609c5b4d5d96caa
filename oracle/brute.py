"""Pure-Python eq. (4) for tiny cases (test infrastructure, oracle).

Used only to pin the C sums: loops over points, positions and frequencies with
``cmath``; no numpy arithmetic.
"""
import cmath
import math

C0 = 299792458.0


def bp_eq4(positions, freqs_hz, echoes, points):
    out = []
    for q in points:
        acc = 0j
        for i, p in enumerate(positions):
            R = math.sqrt((q[0] - p[0]) ** 2 + (q[1] - p[1]) ** 2 + (q[2] - p[2]) ** 2)
            for f, fr in enumerate(freqs_hz):
                k = 2.0 * math.pi * fr / C0
                acc += complex(echoes[i][f]) * cmath.exp(2j * k * R)
        out.append(acc)
    return out


def echoes_eq1(positions, freqs_hz, targets, amps):
    """s(p', k) = sum_t a_t exp(-j 2 k |p_t - p'|), eq. (1)."""
    s = []
    for p in positions:
        row = []
        for fr in freqs_hz:
            k = 2.0 * math.pi * fr / C0
            acc = 0j
            for t, a in zip(targets, amps):
                R = math.sqrt((t[0] - p[0]) ** 2 + (t[1] - p[1]) ** 2 + (t[2] - p[2]) ** 2)
                acc += complex(a) * cmath.exp(-2j * k * R)
            row.append(acc)
        s.append(row)
    return s
