"""Naive one-step evaluator of the coupled LB freezing scheme, written
separately from the C oracle: pure Python, mpmath at 40 digits, one node and
one direction at a time, periodic x by modulo indexing and the wall rules
spelled out per link.  2D only (D2Q9 flow, D2Q5 scalars).  It is a test of
the oracle's implementation (index slips, dropped terms, swapped operands),
following the same readings of the paper's Sec. 3 as the oracle does.
"""
from mpmath import mp, mpf, sqrt, cos, pi

mp.dps = 40

C9 = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
W9 = [mpf(4) / 9] + [mpf(1) / 9] * 4 + [mpf(1) / 36] * 4
C5 = C9[:5]
W5 = [mpf(1) / 3] + [mpf(1) / 6] * 4
CS2 = mpf(1) / 3


def _opp(c, lst):
    return lst.index((-c[0], -c[1]))


def emap(P, E, psi):
    rcs = psi * P["rho_s"] * P["cp_s"] + (1 - psi) * P["rho_g"] * P["cp_g"]
    rcl = psi * P["rho_l"] * P["cp_l"] + (1 - psi) * P["rho_g"] * P["cp_g"]
    Es = rcs * P["T_sol"]
    El = rcl * P["T_liq"] + psi * P["rho_l"] * P["latent"]
    if E < Es:
        fl, T = mpf(0), E / rcs
    elif E > El:
        fl, T = mpf(1), P["T_liq"] + (E - El) / rcl
    else:
        d = El - Es
        fl = mpf(1) if d <= mpf("1e-12") * max(1, abs(E)) else (E - Es) / d
        T = P["T_sol"] + fl * (P["T_liq"] - P["T_sol"])
    return T, psi * (1 - fl)


def prop(phi, fs, zl, zg, zs):
    return phi * (zl - zg) / 2 + fs * (zs - zl) + (zl + zg) / 2


def step(P, pops, state):
    """pops: dict f, g, h, l -> [q][ny][nx] lists of mpf; state: dict fs, p,
    ux, uy, phi, C -> [ny][nx].  Returns (new pops, new state)."""
    P = {k: (mpf(v) if isinstance(v, (int, float)) else v) for k, v in P.items()}
    nx, ny = int(P["nx"]), int(P["ny"])
    rng = [(y, x) for y in range(ny) for x in range(nx)]
    tau_g = P["nu"] / CS2 + mpf(1) / 2
    tau_f, tau_a = P["tau_phi"], P["tau_h"]
    tau_s = tau_a / (2 * tau_a - 1)
    Dl = CS2 * (P["tau_c"] - mpf(1) / 2)
    Ds = P["Ds_over_Dl"] * Dl
    ratio = 1 - P["rho_s"] / P["rho_l"]
    eps = P["eps"]

    def twall(x):
        return P["T_lo"] + P["T_lo_amp"] * cos(2 * pi * x / nx)

    # neighbour with the stencil ghost rules; kind: 's' mirror, 'T' temperature,
    # 'u' negated mirror (no-slip velocity)
    def nb(F, y, x, c, kind):
        xx, yy = (x + c[0]) % nx, y + c[1]
        if 0 <= yy < ny:
            return F[yy][xx]
        if yy < 0:
            m = F[-1 - yy][xx]
            if kind == "T" and P["t_lo_dirichlet"]:
                return 2 * twall(xx) - m
        else:
            m = F[2 * ny - 1 - yy][xx]
            if kind == "T" and P["t_hi_dirichlet"]:
                return 2 * P["T_hi"] - m
        return -m if kind == "u" else m

    def grad(F, y, x, kind):
        gx = sum(W9[i] * C9[i][0] * nb(F, y, x, C9[i], kind) for i in range(1, 9)) / CS2
        gy = sum(W9[i] * C9[i][1] * nb(F, y, x, C9[i], kind) for i in range(1, 9)) / CS2
        return gx, gy

    def lap(F, y, x):
        return sum(2 * W9[i] * (nb(F, y, x, C9[i], "s") - F[y][x]) for i in range(1, 9)) / CS2

    grid = lambda: [[mpf(0)] * nx for _ in range(ny)]
    # divergence of the previous velocity
    D = grid()
    for (y, x) in rng:
        D[y][x] = (grad(state["ux"], y, x, "u")[0] + grad(state["uy"], y, x, "u")[1])
    # closure
    phi, T, C, fs, md, Q, E, rho, rc = (grid() for _ in range(9))
    for (y, x) in rng:
        phi0 = sum(pops["f"][i][y][x] for i in range(5))
        E0 = sum(pops["h"][i][y][x] for i in range(5))
        C[y][x] = sum(pops["l"][i][y][x] for i in range(5))
        psi = min(max((1 + phi0) / 2, mpf(0)), mpf(1))
        ph = phi0 / (1 - D[y][x] / 2)
        T0, fs0 = emap(P, E0, psi)
        q = prop(ph, fs0, P["rho_l"], P["rho_g"], P["rho_s"]) * prop(ph, fs0, P["cp_l"], P["cp_g"], P["cp_s"]) * T0 * D[y][x]
        Ex = E0 + q / 2
        Tn, fsn = emap(P, Ex, psi)
        phi[y][x], T[y][x], fs[y][x], Q[y][x], E[y][x] = ph, Tn, fsn, q, Ex
        md[y][x] = ratio * (fsn - state["fs"][y][x])
        rho[y][x] = prop(ph, fsn, P["rho_l"], P["rho_g"], P["rho_s"])
        rc[y][x] = rho[y][x] * prop(ph, fsn, P["cp_l"], P["cp_g"], P["cp_s"])
    post = {k: [grid() for _ in range(len(pops[k]))] for k in pops}
    new_state = {k: grid() for k in state}
    alpha = 3 * sqrt(2) * eps / 4
    for (y, x) in rng:
        gpx, gpy = grad(phi, y, x, "s")
        gTx, gTy = grad(T, y, x, "T")
        gCx, gCy = grad(C, y, x, "s")
        gfx, gfy = grad(fs, y, x, "s")
        gPx, gPy = grad(state["p"], y, x, "s")
        lp = lap(phi, y, x)
        grx = (P["rho_l"] - P["rho_g"]) / 2 * gpx + (P["rho_s"] - P["rho_l"]) * gfx
        gry = (P["rho_l"] - P["rho_g"]) / 2 * gpy + (P["rho_s"] - P["rho_l"]) * gfy
        ng = sqrt(gpx ** 2 + gpy ** 2)
        den = max(ng, mpf("1e-6"))
        nx_, ny_ = gpx / den, gpy / den
        ph = phi[y][x]
        mu = ph * (ph ** 2 - 1) / eps ** 2 - lp
        sig = P["sigma0"] + P["sigma_T"] * (T[y][x] - P["T_ref"]) + P["sigma_c"] * (C[y][x] - P["c_ref"])
        gsx = P["sigma_T"] * gTx + P["sigma_c"] * gCx
        gsy = P["sigma_T"] * gTy + P["sigma_c"] * gCy
        wst = (1 - fs[y][x]) if int(P["surface_tension_mode"]) == 0 else 1
        Fx = wst * (alpha * sig * mu * gpx + alpha * ((gpx ** 2 + gpy ** 2) * gsx - (gsx * gpx + gsy * gpy) * gpx)) + P["body_force"][0]
        Fy = wst * (alpha * sig * mu * gpy + alpha * ((gpx ** 2 + gpy ** 2) * gsy - (gsx * gpx + gsy * gpy) * gpy)) + P["body_force"][1]
        g = [pops["g"][i][y][x] for i in range(9)]
        r = rho[y][x]
        usx = (sum(C9[i][0] * g[i] for i in range(9)) + Fx / 2) / r
        usy = (sum(C9[i][1] * g[i] for i in range(9)) + Fy / 2) / r
        fdx, fdy = -fs[y][x] * usx, -fs[y][x] * usy
        ux, uy = usx + fdx / 2, usy + fdy / 2
        S = r * md[y][x] + ux * grx + uy * gry
        Ftx = Fx - gPx + CS2 * grx
        Fty = Fy - gPy + CS2 * gry
        G = []
        for i in range(9):
            cx, cy = C9[i]
            # (u Ft + Ft u):(c c - cs2 I), expanded component by component
            A = (2 * ux * Ftx * (cx * cx - CS2) + 2 * uy * Fty * (cy * cy - CS2)
                 + (ux * Fty + uy * Ftx) * 2 * cx * cy)
            G.append(W9[i] * (S + (cx * (Fx + r * fdx) + cy * (Fy + r * fdy)) / CS2 + A / (2 * CS2 ** 2)))
        uu = ux * ux + uy * uy
        s0 = W9[0] * (-uu / (2 * CS2))
        pn = CS2 / (1 - W9[0]) * (sum(g[1:]) + S / 2 + (tau_g - mpf(1) / 2) * G[0] + r * s0)
        for i in range(9):
            cx, cy = C9[i]
            cu = cx * ux + cy * uy
            si = W9[i] * (cu / CS2 + cu * cu / (2 * CS2 ** 2) - uu / (2 * CS2))
            geq = pn / CS2 * ((W9[i] - 1) if i == 0 else W9[i]) + r * si
            post["g"][i][y][x] = g[i] - (g[i] - geq) / tau_g + (1 - 1 / (2 * tau_g)) * G[i]
        # phase field
        Bx = ph * ux - state["phi"][y][x] * state["ux"][y][x] + CS2 * nx_ * (1 - ph * ph) / (sqrt(2) * eps)
        By = ph * uy - state["phi"][y][x] * state["uy"][y][x] + CS2 * ny_ * (1 - ph * ph) / (sqrt(2) * eps)
        for i in range(5):
            cx, cy = C5[i]
            Fi = W5[i] * (cx * Bx + cy * By) / CS2 + W5[i] * ph * D[y][x]
            feq = W5[i] * ph * (1 + (cx * ux + cy * uy) / CS2)
            fi = pops["f"][i][y][x]
            post["f"][i][y][x] = fi - (fi - feq) / tau_f + (1 - 1 / (2 * tau_f)) * Fi
        # enthalpy TRT
        heq = []
        for i in range(5):
            cx, cy = C5[i]
            cu = cx * ux + cy * uy
            if i == 0:
                heq.append(E[y][x] - P["rhoc_ref"] * T[y][x] + W5[0] * (P["rhoc_ref"] * T[y][x] - rc[y][x] * T[y][x] * uu / (2 * CS2)))
            else:
                heq.append(W5[i] * (P["rhoc_ref"] * T[y][x] + rc[y][x] * T[y][x] * (cu / CS2 + (cu * cu - CS2 * uu) / (2 * CS2 ** 2))))
        for i in range(5):
            o = _opp(C5[i], C5)
            hi, ho = pops["h"][i][y][x], pops["h"][o][y][x]
            post["h"][i][y][x] = (hi - ((hi + ho) / 2 - (heq[i] + heq[o]) / 2) / tau_s
                                  - ((hi - ho) / 2 - (heq[i] - heq[o]) / 2) / tau_a
                                  + (1 - 1 / (2 * tau_s)) * W5[i] * Q[y][x])
        # solute
        f_s = fs[y][x]
        keff = 1 - f_s * (1 - P["k_p"])
        tau_l = (f_s * P["k_p"] * Ds + (1 - f_s) * Dl) / (CS2 * keff) + mpf(1) / 2
        Cc = C[y][x]
        Rx = (1 - ph) * Cc * nx_ / (sqrt(2) * eps) + (P["k_p"] - 1) * Cc * gfx / keff
        Ry = (1 - ph) * Cc * ny_ / (sqrt(2) * eps) + (P["k_p"] - 1) * Cc * gfy / keff
        Lx = Cc * ux - state["C"][y][x] * state["ux"][y][x] + CS2 * Rx
        Ly = Cc * uy - state["C"][y][x] * state["uy"][y][x] + CS2 * Ry
        for i in range(5):
            cx, cy = C5[i]
            Li = W5[i] * (cx * Lx + cy * Ly) / CS2
            leq = W5[i] * Cc * (1 + (cx * ux + cy * uy) / CS2)
            li = pops["l"][i][y][x]
            post["l"][i][y][x] = li - (li - leq) / tau_l + (1 - 1 / (2 * tau_l)) * Li
        new_state["fs"][y][x] = f_s
        new_state["p"][y][x] = pn
        new_state["ux"][y][x] = ux
        new_state["uy"][y][x] = uy
        new_state["phi"][y][x] = ph
        new_state["C"][y][x] = Cc
    # streaming: push every post-collision population along its link
    new = {k: [grid() for _ in range(len(pops[k]))] for k in pops}
    for k, lst in (("f", C5), ("g", C9), ("h", C5), ("l", C5)):
        for (y, x) in rng:
            for i, c in enumerate(lst):
                val = post[k][i][y][x]
                tx, ty = (x + c[0]) % nx, y + c[1]
                if 0 <= ty < ny:
                    new[k][i][ty][tx] = val
                    continue
                o = _opp(c, lst)          # bounced back into the same node
                if k == "h" and ty < 0 and P["t_lo_dirichlet"]:
                    val = -val + 2 * W5[o] * P["rhoc_ref"] * twall(x)
                elif k == "h" and ty >= ny and P["t_hi_dirichlet"]:
                    val = -val + 2 * W5[o] * P["rhoc_ref"] * P["T_hi"]
                new[k][o][y][x] = val
    return new, new_state
