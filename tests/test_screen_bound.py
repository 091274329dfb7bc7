"""The certification rule of the phase-cell kernel's FP32 screen (Eq. 7 ownership), in exact
arithmetic on the CPU.

The kernel forms, per (incoming direction, lattice point) pair, the rotated point in FP32
(q'_k = fma(R_2k', p_2', fma(R_1k', p_1', R_0k' p_0')) from the FP32 roundings of the FP64
rotation R and lattice point p), then for each out-edge m
    t_m = fma(q2', s_m2', fma(q1', s_m1', fma(q0', s_m0', 1 + 2^-10)))
with s' the FP32 rounding of the FP64 unit direction, packs 63 - m into the low six bits of
t_m and keeps the largest and second largest packed values.  It trusts the packed argmax b
only if  best - second > fma(best, 2^-16, 2^-17)  (all FP32).  Its stated error bound
implies that a trusted b beats every other out-edge by more than 2^-50 in exact arithmetic
on the FP64 inputs, so any FP64 evaluation within 2^-51 (the kernel's FP64 sequence) takes
the same argmax with no tie.  This test emulates every FP32 operation with correct
rounding (exact rationals) on stencils built to have near-ties, and checks that conclusion
for each certified pair, and that the screen certifies almost every pair of a jittered grid.
"""
import math
from fractions import Fraction as Fr

import numpy as np


def f32(x: Fr) -> Fr:
    """x rounded to the nearest FP32 value (ties to even), as an exact rational."""
    if x == 0:
        return Fr(0)
    c = np.float32(float(x))  # within one ulp of the correct rounding
    best = None
    for cand in (np.nextafter(c, np.float32(-np.inf)), c, np.nextafter(c, np.float32(np.inf))):
        cf = Fr(float(cand))
        key = (abs(cf - x), int(np.float32(cand).view(np.uint32)) & 1)
        if best is None or key < best[0]:
            best = (key, cf)
    return best[1]


def fma(a, b, c):
    return f32(a * b + c)


def pack(t: Fr, k: int) -> Fr:
    bits = int(np.float32(float(t)).view(np.uint32))  # t is an exact FP32 value here
    return Fr(float(np.uint32((bits & ~63) | k).view(np.float32)))


def lattice(n):
    ga = math.pi * (3.0 - math.sqrt(5.0))
    out = []
    for i in range(n):
        z = 1.0 - (2.0 * i + 1.0) / n
        ph = math.fmod(i * ga, 2.0 * math.pi)
        r = math.sqrt(1.0 - z * z)
        out.append((r * math.cos(ph), r * math.sin(ph), z))
    return out


def rotation(u):
    ux, uy, uz = u
    h = 1.0 / (1.0 + uz)
    xy = (ux * uy) * h
    return [[uz + (uy * uy) * h, -xy, -ux], [-xy, uz + (ux * ux) * h, -uy], [ux, uy, uz]]


def unit(D):
    n = math.sqrt(float(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]))
    return (D[0] / n, D[1] / n, D[2] / n)


def screen(R, p, sites):
    """The kernel's FP32 screen for one pair: (packed argmax, certified)."""
    Rq = [[Fr(R[r][k]) for k in range(3)] for r in range(3)]
    c = [[f32(Rq[r][k]) for r in range(3)] for k in range(3)]  # columns of R in FP32
    pt = [f32(Fr(x)) for x in p]
    q = [fma(c[k][2], pt[2], fma(c[k][1], pt[1], f32(c[k][0] * pt[0]))) for k in range(3)]
    off = f32(Fr(1) + Fr(1, 1024))
    best = second = Fr(0)
    for m, s in enumerate(sites):
        sf = [f32(Fr(x)) for x in s]
        t = fma(q[2], sf[2], fma(q[1], sf[1], fma(q[0], sf[0], off)))
        v = pack(t, 63 - m)
        if v > best:
            best, second = v, best
        elif v > second:
            second = v
    b = 63 - (int(np.float32(float(best)).view(np.uint32)) & 63)
    cert = f32(best - second) > fma(best, Fr(1, 2 ** 16), Fr(1, 2 ** 17))
    return b, cert


def exact_gaps(R, p, sites, b):
    """Exact q.s_b - q.s_m for m != b, q = R^T p on the FP64 values."""
    q = [sum(Fr(R[r][k]) * Fr(p[r]) for r in range(3)) for k in range(3)]
    v = [sum(q[k] * Fr(s[k]) for k in range(3)) for s in sites]
    return [v[b] - v[m] for m in range(len(sites)) if m != b]


def check(sites, dirs, pts):
    n_cert = n = 0
    for u in dirs:
        R = rotation(u)
        for p in pts:
            b, cert = screen(R, p, sites)
            n += 1
            if cert:
                n_cert += 1
                assert min(exact_gaps(R, p, sites, b)) > Fr(1, 2 ** 50), (u, p, b)
    return n_cert, n


def test_certified_owners_win_by_more_than_the_fp64_error():
    rng = np.random.default_rng(7)
    F = 65536
    # near-duplicate out-edges (integer offsets a few fixed-point units apart: directions
    # 1e-6 .. 1e-4 rad apart) at distant indices, so that packing the index alone could
    # reorder them; exact mirror pairs and a jittered shell
    head = [(F, 0, 0), (-F, 0, 0), (0, F, 0), (0, 0, F), (0, 0, -F), (F, F, 0), (F, -F, 0), (-F, F, F)]
    jit = [tuple(int(x) for x in rng.integers(-2 * F, 2 * F, 3)) for _ in range(10)]
    tail = [(F, 3, 0), (F, 0, 7), (0, F, 1), (F, F, 2), (-F, F, F + 5), (1, 2, F)]
    sites = [unit(D) for D in head + jit + tail]
    near = [(0, 18), (0, 19), (2, 20), (5, 21), (7, 22), (3, 23)]
    dirs = [tuple(-x for x in sites[a]) for a in (0, 2, 5, 7)] + [unit((3, -2, -9))]
    lat = lattice(100)
    pts = [lat[i] for i in rng.choice(100, 16, replace=False)]
    # lattice points on the bisector of two nearly equal out-edges (the hardest ties), and
    # points a few 1e-7 rad off it toward the later index (whose true value then wins)
    for a, b in near:
        sa, sb = np.array(sites[a]), np.array(sites[b])
        for eps in (0.0, 2e-7, 1e-6, 5e-6):
            v = sa + sb + eps * (sb - sa) / max(np.linalg.norm(sb - sa), 1e-300)
            pts.append(tuple(v / np.linalg.norm(v)))
    n_cert, n = check(sites, dirs, pts)
    assert n_cert > 0 and n_cert < n  # both outcomes occur on this stencil


def test_screen_certifies_almost_every_pair_of_a_jittered_stencil():
    rng = np.random.default_rng(3)
    F = 65536
    offs = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1) if (dx, dy, dz) != (0, 0, 0)]
    sites = [unit(tuple(int(F * o + j) for o, j in zip(D, rng.integers(-F // 4, F // 4, 3)))) for D in offs[:22]]
    dirs = [tuple(-x for x in sites[a]) for a in (0, 7)]
    pts = lattice(100)[::4]
    n_cert, n = check(sites, dirs, pts)
    assert n_cert >= n - 1
