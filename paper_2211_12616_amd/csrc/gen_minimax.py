"""Coefficients of the FP64 polynomials in mpt_math.h.

Each polynomial is the weighted minimax approximation (Remez exchange in
50-digit arithmetic) of the smooth remainder of a series, on the range the
step kernels feed it, rounded to the nearest double:

* ln:   q(z) ~ (atanh(s)/s - 1)/z,  z = s^2 in [0, ((sqrt2-1)/(sqrt2+1))^2];
        ln m = 2s + 2s z q(z), so the error of q counts as z * dq relative.
* sin:  h(z) ~ (sin(x)/x - 1)/z,    z = x^2 in [0, (pi/2 + 0.02)^2]
        (cos of a latitude as the sine of the co-latitude, with a small
        overshoot past the poles) and in [0, (pi/4)^2] (sin(pi t) after the
        reduction by quarter periods); sin x = x + x z h(z), so the error of h
        counts as z * dh relative.
* cos:  g(z) ~ (cos(x) - 1 + z/2)/z^2, z in [0, (pi/4)^2];
        cos x = 1 - z/2 + z^2 g(z), so the error of g counts as z^2 * dg.

Run with mpmath available: python gen_minimax.py.  It prints, per
polynomial, the weighted error before and after rounding the coefficients
and the coefficients from the highest power down, as C hex literals.
"""
import mpmath as mp

mp.mp.dps = 50


def remez(f, a, b, deg, w, iters=12, grid_n=4000):
    n = deg + 2
    xs = [(a + b) / 2 - (b - a) / 2 * mp.cos(mp.pi * i / (n - 1)) for i in range(n)]
    grid = [a + (b - a) * mp.mpf(k) / grid_n for k in range(grid_n + 1)]
    for _ in range(iters):
        A = mp.matrix(n, n)
        rhs = mp.matrix(n, 1)
        for i, x in enumerate(xs):
            for j in range(deg + 1):
                A[i, j] = x ** j
            A[i, deg + 1] = (-1) ** i / w(x)
            rhs[i] = f(x)
        sol = mp.lu_solve(A, rhs)
        c = [sol[j] for j in range(deg + 1)]
        vals = [w(x) * (mp.polyval(c[::-1], x) - f(x)) for x in grid]
        ext, run = [], [0]
        for k in range(1, len(grid)):
            if (vals[k] >= 0) == (vals[run[0]] >= 0):
                run.append(k)
            else:
                ext.append(max(run, key=lambda t: abs(vals[t])))
                run = [k]
        ext.append(max(run, key=lambda t: abs(vals[t])))
        while len(ext) > n:
            ext.pop(0 if abs(vals[ext[0]]) < abs(vals[ext[-1]]) else -1)
        if len(ext) < n:
            break
        xs = [grid[k] for k in ext]
    return c, max(abs(v) for v in vals)


def weighted_err(f, a, b, coefs, w, grid_n=20000):
    cm = [mp.mpf(v) for v in coefs[::-1]]
    return max(abs(w(x) * (mp.polyval(cm, x) - f(x)))
               for x in (a + (b - a) * mp.mpf(k) / grid_n for k in range(grid_n + 1)))


def q_ln(z):
    if z == 0:
        return mp.mpf(1) / 3
    s = mp.sqrt(z)
    return (mp.atanh(s) / s - 1) / z


def h_sin(z):
    if z == 0:
        return mp.mpf(-1) / 6
    x = mp.sqrt(z)
    return (mp.sin(x) / x - 1) / z


def g_cos(z):
    if z == 0:
        return mp.mpf(1) / 24
    x = mp.sqrt(z)
    return (mp.cos(x) - 1 + z / 2) / (z * z)


def main():
    zln = ((mp.sqrt(2) - 1) / (mp.sqrt(2) + 1)) ** 2 * mp.mpf("1.0001")
    zlat = (mp.pi / 2 + mp.mpf("0.02")) ** 2
    zq = (mp.pi / 4) ** 2 * mp.mpf("1.0002")
    # weights: the relative error each polynomial adds to its function (a
    # small floor keeps the exchange well posed at z = 0)
    jobs = [
        ("ln q", q_ln, zln, 6, lambda z: z + zln / 1000),
        ("sin h, to pi/2", h_sin, zlat, 7, lambda z: z + mp.mpf("0.0025")),
        ("sin h, to pi/4", h_sin, zq, 5, lambda z: z + mp.mpf("0.0006")),
        ("cos g, to pi/4", g_cos, zq, 5, lambda z: z * z + mp.mpf("1e-6")),
    ]
    for name, f, b, deg, w in jobs:
        c, e = remez(f, mp.mpf(0), b, deg, w)
        cd = [float(v) for v in c]
        ed = weighted_err(f, mp.mpf(0), b, cd, w)
        print(f"{name}: degree {deg}, weighted error {mp.nstr(e, 3)}, "
              f"{mp.nstr(ed, 3)} with double coefficients")
        for v in cd[::-1]:
            print("   ", v.hex())


if __name__ == "__main__":
    main()
