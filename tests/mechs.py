"""Hand-built tiny mechanisms used by the pins (test helpers, no kinetics)."""
import numpy as np


def nasa_row(a1, a6, a7, a2=0.0, a3=0.0, a4=0.0, a5=0.0, tmid=1000.0):
    row = [a1, a2, a3, a4, a5, a6, a7]
    return np.array([tmid] + row + row, dtype=np.float64)


def base(K, R, comps, W, nasa):
    return dict(n_species=K, n_reactions=R, n_elements=4, W=np.asarray(W, np.float64),
                nasa7=np.asarray(nasa, np.float64), elem=np.asarray(comps, np.int32),
                rtype=np.zeros(R, np.int32), reac=-np.ones((R, 3), np.int32),
                prod=-np.ones((R, 3), np.int32), lnA=np.zeros(R), b=np.zeros(R),
                theta=np.zeros(R), eff=np.ones((R, K)), troe=np.zeros((R, 4)),
                low=np.zeros((R, 3)))


def isomer_mech(kind="elementary", A=1e6, b=0.5, theta=3000.0, n_inert=1):
    """Species A, B (isomers with identical thermo) and n_inert copies of an
    inert I; one reaction.

    kind: "elementary" (A <=> B), "thirdbody" (A + M <=> B + M, unit
    efficiencies) or "troe" (A (+M) <=> B (+M)).  K_c = 1 and the reaction is
    thermoneutral, so T stays constant and Y_A - Y_B decays as exp(-2 k t).
    """
    comps = [[1, 2, 0, 0], [1, 2, 0, 0]] + [[0, 0, 0, 2]] * n_inert
    W = [14.027, 14.027] + [28.014] * n_inert
    nasa = [nasa_row(4.0, -1000.0, 5.0, a2=1e-3), nasa_row(4.0, -1000.0, 5.0, a2=1e-3)] + \
        [nasa_row(3.5, -500.0, 4.0)] * n_inert
    m = base(2 + n_inert, 1, comps, W, nasa)
    m["reac"][0, 0] = 0
    m["prod"][0, 0] = 1
    m["lnA"][0], m["b"][0], m["theta"][0] = np.log(A), b, theta
    if kind == "thirdbody":
        m["rtype"][0] = 1
    elif kind == "troe":
        m["rtype"][0] = 2
        m["troe"][0] = [0.6, 100.0, 1500.0, 4000.0]
        m["low"][0] = [np.log(A) + np.log(10.0) * 4.0, -1.0, 0.5 * theta]
    return m


def lindemann_mech():
    """One Troe reaction whose broadening factor is exactly 1 (F_cent = 1)."""
    m = isomer_mech("troe")
    # alpha = 1 keeps only exp(-T/T*) with T* -> huge (=1) and exp(-T**/T) with T** -> huge (=0)
    m["troe"][0] = [1.0, 100.0, 1e300, 1e300]
    return m
