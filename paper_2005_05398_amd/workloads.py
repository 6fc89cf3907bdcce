"""Problem descriptions and seeded inputs shared by the oracle tests, the HIP
path's tests and the benchmark.

This module holds data only: particle sets, grid sizes, domains, energies and
seeded random right-hand sides.  It contains none of the method's arithmetic,
so both sides of every parity test can take their inputs from here without
sharing code.

A problem description is a plain dict:

    masses   (m1, m2, m3)              particle masses (Sec. 2.1)
    charges  (Z1, Z2, Z3)              particle charges (Sec. 2.1)
    J, tau                             total orbital momentum and parity (Sec. 2.2)
    x, y, z  [dim, dim, dim]           one 1D basis per Faddeev component alpha
             dim = {"degree": 3|5, "n": int, "R": float, "map": str}
    x0, y0, nu                         Merkuriev cut-off parameters, eq. (Mcutoff0)
    vhat                               0: Vhat_a(y) = Z_a(Z_b+Z_c) sqrt(2 mu_a(bc)) / (y+1)

"map" is "uniform" or "quadratic" for x, y and "sin" or "uniform" for z.
"""
import math

import numpy as np

INF = math.inf


def _dims(degree, n, R, mapname):
    return [{"degree": degree, "n": n, "R": R, "map": mapname} for _ in range(3)]


def make_desc(masses, charges, nxy, nz, *, J=0, tau=1, deg_xy=5, deg_z=5,
              R=20.0, xy_map="uniform", z_map="sin", x0=5.0, y0=INF, nu=2.01,
              vhat=0):
    """A description with the same grid for all three components."""
    return {
        "masses": tuple(float(m) for m in masses),
        "charges": tuple(float(c) for c in charges),
        "J": int(J), "tau": int(tau),
        "x": _dims(deg_xy, nxy, R, xy_map),
        "y": _dims(deg_xy, nxy, R, xy_map),
        "z": _dims(deg_z, nz, 2.0, z_map),
        "x0": float(x0), "y0": float(y0), "nu": float(nu), "vhat": int(vhat),
    }


def admissible_xy(n, degree=5):
    """Nearest admissible x/y basis size: quintic n = 3K+1, cubic n = 2K."""
    if degree == 3:
        return n + (n % 2)
    cands = [m for m in range(max(4, n - 3), n + 4) if m % 3 == 1]
    return min(cands, key=lambda m: (abs(m - n), m))


# Particle sets of the workloads.
PS_MINUS = ((1.0, 1.0, 1.0), (1.0, -1.0, -1.0))       # e+ e- e- : particles 2, 3 identical
H_MINUS = ((1.0, 1.0, 1836.0), (-1.0, -1.0, 1.0))     # e- e- p  : particles 1, 2 identical


def ps_cubic16():
    """FP64, L=0, cubic 16 x 16 x 8 on [0,20]^2 x [-1,1], E=-0.25, one RHS."""
    d = make_desc(*PS_MINUS, 16, 8, deg_xy=3, deg_z=3, R=20.0)
    return {"name": "ps_cubic_16x16x8_L0", "desc": d, "E": [-0.25], "seeds": [1001]}


def hminus_scan():
    """FP64, L=0, quintic 64 x 64 x 24, x,y in [0,40] graded quadratically
    toward 0, energy scan of 32 values in [-0.6, -0.1], one RHS per energy."""
    d = make_desc(*H_MINUS, 64, 24, deg_xy=5, deg_z=5, R=40.0, xy_map="quadratic")
    E = list(np.linspace(-0.6, -0.1, 32))
    return {"name": "hminus_quintic_64x64x24_L0_scan32", "desc": d, "E": E,
            "seeds": [2001 + i for i in range(32)]}


def ps_q127():
    """Mixed precision, L=0, quintic x,y (nominal 128, taken as 127 = 3*42+1,
    uniform on [0,20]) x cubic z 32."""
    d = make_desc(*PS_MINUS, admissible_xy(128), 32, deg_xy=5, deg_z=3, R=20.0)
    return {"name": "ps_quintic127_cubicz32_L0", "desc": d, "E": [-0.25], "seeds": [3001]}


def ps_l2_q97():
    """L=2, tau=+1 (three M' blocks), quintic x,y (nominal 96, taken as
    97 = 3*32+1) x cubic z 32, E=-0.2."""
    d = make_desc(*PS_MINUS, admissible_xy(96), 32, J=2, tau=1, deg_xy=5, deg_z=3, R=20.0)
    return {"name": "ps_L2_quintic97_cubicz32", "desc": d, "E": [-0.2], "seeds": [4001]}


def pair_pair_desc(nz=4, deg_z=3):
    """A small Ps- like L=0 grid (quintic x 43 on [0,30], y 19 on [0,24],
    uniform) on which one preconditioner slice of component 1 has complex
    eigenvalue pairs in both its x and its y pencil, so that the divide meets
    the 4 x 4 real blocks of an x pair against a y pair (no workload grid
    has them)."""
    d = make_desc(*PS_MINUS, 43, nz, deg_xy=5, deg_z=deg_z, R=30.0)
    d["y"] = make_desc(*PS_MINUS, 19, nz, deg_xy=5, deg_z=deg_z, R=24.0)["y"]
    return d


WORKLOADS = {"ps_cubic16": ps_cubic16, "hminus_scan": hminus_scan, "ps_q127": ps_q127, "ps_l2_q97": ps_l2_q97}


# Helium with an infinitely heavy nucleus (1e15 a.u.), the runs of Sec. 4:
# quintic splines, x and y nodes by eq. (map-pow), z nodes sin(pi u / 2),
# Merkuriev cut-off x0 = 1, nu = 2.01, y0 = infinity.  Particles 1, 2 are the
# electrons and 3 the nucleus, so components 1 and 2 hold an electron-nucleus
# pair and component 3 the electron pair.  The paper's domain lengths are
# distances in the unscaled Jacobi vectors: a box length R of x_alpha (y_alpha)
# becomes R sqrt(2 mu) in the mass-scaled coordinates the equations use, mu
# the pair's (the third particle's) reduced mass.
HE_MASSES = (1.0, 1.0, 1e15)
HE_CHARGES = (-1.0, -1.0, 2.0)

# Table 1 of Sec. 4 (the comparison with Pardiso; J = 1, tau = +1; domains
# (1: 36, 36; 3: 9, 6)): basis sizes of components (1, 3) as (n_x, n_y, n_z)
# and the printed 2 1P and 3 1P energies; the benchmark values the caption
# quotes.
HE_TABLE1 = [((22, 22, 9), (19, 19, 12), (-2.12524, -2.05654)),
             ((31, 31, 9), (22, 22, 15), (-2.12365, -2.05495)),
             ((40, 40, 12), (25, 25, 18), (-2.12378, -2.05508)),
             ((49, 49, 12), (28, 28, 21), (-2.12385, -2.05513)),
             ((58, 58, 12), (28, 28, 21), (-2.12384, -2.05514))]
HE_TABLE1_DOMAINS = ((36.0, 36.0), (9.0, 6.0))
HE_1P_BENCHMARK = (-2.12384308649810135925, -2.05514636209194353689)

# Table 3 of Sec. 4 (the high-J runs: J = 10, tau = +1, p = +1, eleven M'
# blocks; domains (1: 280, 280; 3: 2, 2)): basis sizes of components (1, 3)
# and the printed ground and first excited energies.
HE_TABLE3_J10 = [((58, 58, 6), (4, 4, 6), (-2.00398, -2.00332)),
                 ((88, 88, 9), (7, 7, 9), (-2.00412, -2.00346)),
                 ((118, 118, 9), (7, 7, 9), (-2.00413, -2.00347)),
                 ((118, 118, 12), (7, 7, 12), (-2.00413, -2.00347))]
HE_TABLE3_DOMAINS = ((280.0, 280.0), (2.0, 2.0))


def helium_desc(g1, g3, dom1=HE_TABLE1_DOMAINS[0], dom3=HE_TABLE1_DOMAINS[1], J=1, tau=1):
    """Helium description with basis sizes g1 (components 1, 2) and g3
    (component 3), each (n_x, n_y, n_z), on the paper's domains (unscaled
    lengths, see above)."""
    m = HE_MASSES
    M = sum(m)
    dims = {"x": [], "y": [], "z": []}
    for a in range(3):
        b, c = [i for i in range(3) if i != a]
        mu_x = m[b] * m[c] / (m[b] + m[c])
        mu_y = m[a] * (m[b] + m[c]) / M
        g, dom = (g3, dom3) if a == 2 else (g1, dom1)
        dims["x"].append({"degree": 5, "n": g[0], "R": dom[0] * math.sqrt(2.0 * mu_x), "map": "pow"})
        dims["y"].append({"degree": 5, "n": g[1], "R": dom[1] * math.sqrt(2.0 * mu_y), "map": "pow"})
        dims["z"].append({"degree": 5, "n": g[2], "R": 2.0, "map": "sin"})
    return {"masses": HE_MASSES, "charges": HE_CHARGES, "J": int(J), "tau": int(tau), **dims,
            "x0": 1.0, "y0": INF, "nu": 2.01, "vhat": 0}


def serving_request(i):
    """Request i of the serving stream (seed 5001 + i): nominal x,y size in
    {32, 64, 96, 128} (quintic, taken to the nearest 3K+1), cubic z in
    {8, 16, 32}, L in {0, 1, 2} with tau = +1, E uniform in [-0.6, -0.05], and
    one of the two particle sets with its own domain and map."""
    rr = np.random.Generator(np.random.PCG64(5001 + i))
    nxy = int(rr.choice([32, 64, 96, 128]))
    nz = int(rr.choice([8, 16, 32]))
    L = int(rr.choice([0, 1, 2]))
    E = float(rr.uniform(-0.6, -0.05))
    heavy = bool(rr.integers(2))
    if heavy:
        mc, R, xy_map = H_MINUS, 40.0, "quadratic"
    else:
        mc, R, xy_map = PS_MINUS, 20.0, "uniform"
    desc = make_desc(*mc, admissible_xy(nxy), nz, J=L, tau=1, deg_xy=5, deg_z=3, R=R, xy_map=xy_map)
    return {"desc": desc, "E": E, "seed": 5001 + i, "nominal": {"nxy": nxy, "nz": nz, "L": L, "heavy": heavy}}


def serving_arrivals(n, rate):
    """Poisson arrival times (seconds from start) of n requests at `rate` per second."""
    gaps = np.random.Generator(np.random.PCG64(5000)).exponential(1.0 / rate, n)
    return np.cumsum(gaps) - gaps[0]


def n_unknowns(desc):
    """N = n_M * sum_alpha n_z n_x n_y with n_M = J - M0 + 1, M0 = (1 - tau)/2
    (components 1 and 3 only with the exchange symmetry of two identical
    particles, exchange = +-1; component 1 only for three, exchange = 3)."""
    m0 = (1 - desc["tau"]) // 2
    n_m = desc["J"] - m0 + 1
    ex = desc.get("exchange", 0)
    comps = (0,) if ex == 3 else (0, 2) if ex else (0, 1, 2)

    def nz(a):
        z = desc["z"][a]
        if not (a == 2 and desc.get("zhalf", 0)):
            return z["n"]
        # component 3 on z in [0, 1]: parity sigma = p (-1)^{M0} at z = 0
        if z["degree"] == 3:
            return z["n"] // 2
        K = z["n"] // 3 - 1
        sigma = ex * (-1) ** m0
        return 3 * K // 2 + (2 if sigma == 1 else 1)
    return n_m * sum(nz(a) * desc["x"][a]["n"] * desc["y"][a]["n"] for a in comps)


def rhs(seed, n):
    """Seeded N(0,1) right-hand side in collocation-row space (PCG64)."""
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(n)


def rhs_batch(seeds, n):
    return np.stack([rhs(s, n) for s in seeds])
