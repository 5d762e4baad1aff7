"""Pure-Python brute-force step for tiny lattices (<= 8x8).

An implementation of the same step written independently of the C oracle:
no arrays of planes, no shared tables; plain nested lists and explicit loops.
Used only to cross-check the oracle on random states.

State layout: f[s][y][x][i] for component s in (0, 1) and link i in 0..8,
g[y][x][k] for k in 0..4, solid[y][x] in {0, 1}, m[y][x].
"""

from __future__ import annotations

import copy

LINKS = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
WEIGHT = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
WEIGHT5 = [1 / 3] + [1 / 6] * 4


def reverse(i: int) -> int:
    ex, ey = LINKS[i]
    return LINKS.index((-ex, -ey))


def step(state: dict, prm: dict) -> dict:
    """Advance one step.  prm keys: tau, G, Gads (pair), tau_g, k_r, thr, ax, ay."""
    f, g, solid, m = state["f"], state["g"], state["solid"], state["m"]
    ny, nx = len(solid), len(solid[0])
    tau, tg = prm["tau"], prm["tau_g"]

    def at(y, x):
        return y % ny, x % nx

    rho = [[[0.0] * nx for _ in range(ny)] for _ in range(2)]
    mom = [[[(0.0, 0.0)] * nx for _ in range(ny)] for _ in range(2)]
    conc = [[0.0] * nx for _ in range(ny)]
    for y in range(ny):
        for x in range(nx):
            if solid[y][x]:
                continue
            for s in range(2):
                rho[s][y][x] = sum(f[s][y][x])
                mom[s][y][x] = (sum(f[s][y][x][i] * LINKS[i][0] for i in range(9)),
                                sum(f[s][y][x][i] * LINKS[i][1] for i in range(9)))
            conc[y][x] = sum(g[y][x]) if tg > 0 else 0.0

    post = [[[None] * nx for _ in range(ny)] for _ in range(2)]
    gpost = [[None] * nx for _ in range(ny)]
    m_new = copy.deepcopy(m)
    for y in range(ny):
        for x in range(nx):
            if solid[y][x]:
                continue
            force = []
            for s in range(2):
                other = 1 - s
                coh = [0.0, 0.0]
                adh = [0.0, 0.0]
                for i in range(1, 9):
                    yy, xx = at(y + LINKS[i][1], x + LINKS[i][0])
                    for d in range(2):
                        coh[d] += WEIGHT[i] * rho[other][yy][xx] * LINKS[i][d]
                        adh[d] += WEIGHT[i] * solid[yy][xx] * LINKS[i][d]
                r = rho[s][y][x]
                acc = (prm["ax"], prm["ay"])
                force.append([-prm["G"] * r * coh[d] - prm["Gads"][s] * r * adh[d] + r * acc[d]
                              for d in range(2)])
            rtot = rho[0][y][x] + rho[1][y][x]
            ucommon = [(mom[0][y][x][d] + mom[1][y][x][d]) / rtot for d in range(2)]
            for s in range(2):
                r = rho[s][y][x]
                v = list(ucommon)
                if r > 0:
                    v = [ucommon[d] + tau * force[s][d] / r for d in range(2)]
                out = []
                for i in range(9):
                    eu = LINKS[i][0] * v[0] + LINKS[i][1] * v[1]
                    eq = WEIGHT[i] * r * (1 + 3 * eu + 4.5 * eu * eu
                                          - 1.5 * (v[0] * v[0] + v[1] * v[1]))
                    out.append(f[s][y][x][i] - (f[s][y][x][i] - eq) / tau)
                post[s][y][x] = out
            if tg > 0:
                u = [(mom[0][y][x][d] + mom[1][y][x][d]
                      + 0.5 * (force[0][d] + force[1][d])) / rtot for d in range(2)]
                c = conc[y][x]
                gp = []
                for k in range(5):
                    eq = WEIGHT5[k] * c * (1 + 3 * (LINKS[k][0] * u[0] + LINKS[k][1] * u[1]))
                    gp.append(g[y][x][k] - (g[y][x][k] - eq) / tg)
                if prm["k_r"] > 0:
                    walls = 0
                    for k in range(1, 5):
                        yy, xx = at(y + LINKS[k][1], x + LINKS[k][0])
                        walls += solid[yy][xx]
                    if walls:
                        rate = prm["k_r"] * walls * rho[0][y][x] / rtot
                        m_new[y][x] += rate * c
                        gp = [q * (1 - rate) for q in gp]
                gpost[y][x] = gp

    f_new = [[[[0.0] * 9 for _ in range(nx)] for _ in range(ny)] for _ in range(2)]
    g_new = [[[0.0] * 5 for _ in range(nx)] for _ in range(ny)]
    for y in range(ny):
        for x in range(nx):
            if solid[y][x]:
                continue
            for i in range(9):
                yy, xx = at(y - LINKS[i][1], x - LINKS[i][0])
                for s in range(2):
                    if solid[yy][xx]:
                        f_new[s][y][x][i] = post[s][y][x][reverse(i)]
                    else:
                        f_new[s][y][x][i] = post[s][yy][xx][i]
            if tg > 0:
                for k in range(5):
                    yy, xx = at(y - LINKS[k][1], x - LINKS[k][0])
                    g_new[y][x][k] = gpost[y][x][reverse(k)] if solid[yy][xx] else gpost[yy][xx][k]

    solid_new = copy.deepcopy(solid)
    events = []
    removed = list(state.get("removed", [0.0, 0.0, 0.0]))
    if prm["k_r"] > 0:
        for y in range(ny):
            for x in range(nx):
                if not solid[y][x] and m_new[y][x] > prm["thr"]:
                    solid_new[y][x] = 1
                    removed[0] += sum(f_new[0][y][x])
                    removed[1] += sum(f_new[1][y][x])
                    removed[2] += sum(g_new[y][x])
                    f_new[0][y][x] = [0.0] * 9
                    f_new[1][y][x] = [0.0] * 9
                    g_new[y][x] = [0.0] * 5
                    events.append((x, y, state["step"] + 1))
    return {"f": f_new, "g": g_new, "solid": solid_new, "m": m_new,
            "step": state["step"] + 1, "events": state.get("events", []) + events,
            "removed": removed}
