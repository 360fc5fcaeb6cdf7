"""Naive one-step evaluator of the 3D coupled LB freezing scheme (D3Q19 flow,
D3Q7 phase field, enthalpy and solute), written separately from the C oracle:
pure Python, mpmath at 40 digits, one node and one direction at a time, x
and y periodic by modulo indexing, walls on z at -1/2 and nz - 1/2, and the
rules of a fixed obstacle spelled out per link.  It tests the oracle's 3D
implementation (ghost values at the walls, the edge links of D3Q19 at a
wall, every obstacle rule) under the same readings of the paper's Sec. 3 as
the oracle:

* stencil ghosts across a wall: mirror for phi, C, f_s, p; 2 T_w - T at a
  Dirichlet wall, mirror at an adiabatic one; the negated mirror velocity
  (no slip);
* an obstacle neighbour in the phi, C, f_s, p stencils takes the centre
  node's value, in the velocity divergence the negated centre velocity; the
  obstacle conducts heat (its own T in the T stencil);
* an obstacle node: phi = -1, C = 0, no phase-change material (psi = 0), at
  rest, p = 0; its enthalpy relaxes (TRT) without source; f, g, l vanish;
* streaming: half-way bounce-back at walls and at obstacle links for f, g,
  l; anti-bounce-back for h at a Dirichlet wall; h streams through
  obstacles.
"""
from mpmath import mp, mpf, sqrt, cos, pi

mp.dps = 40

C7 = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
C19 = C7 + [(1, 1, 0), (1, -1, 0), (-1, 1, 0), (-1, -1, 0),
            (1, 0, 1), (1, 0, -1), (-1, 0, 1), (-1, 0, -1),
            (0, 1, 1), (0, 1, -1), (0, -1, 1), (0, -1, -1)]
W7 = [mpf(0)] + [mpf(1) / 6] * 6
W19 = [mpf(1) / 3] + [mpf(1) / 18] * 6 + [mpf(1) / 36] * 12
CS2 = mpf(1) / 3


def _opp(c, lst):
    return lst.index((-c[0], -c[1], -c[2]))


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


def dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def step(P, pops, state, mask):
    """pops: dict f, g, h, l -> [q][nz][ny][nx] nested lists of mpf; state:
    dict fs, p, ux, uy, uz, phi, C -> [nz][ny][nx]; mask: [nz][ny][nx] of
    0 / 1.  Returns (new pops, new state)."""
    P = {k: (mpf(v) if isinstance(v, (int, float)) else v) for k, v in P.items()}
    nx, ny, nz = int(P["nx"]), int(P["ny"]), int(P["nz"])
    nodes = [(z, y, x) for z in range(nz) for y in range(ny) for x in range(nx)]
    tau_g = P["nu"] / CS2 + mpf(1) / 2
    tau_f, tau_a = P["tau_phi"], P["tau_h"]
    tau_s = tau_a / (2 * tau_a - 1)
    Dl = CS2 * (P["tau_c"] - mpf(1) / 2)
    Ds = P["Ds_over_Dl"] * Dl
    ratio = 1 - P["rho_s"] / P["rho_l"]
    eps = P["eps"]
    isq = 1 / (sqrt(2) * eps)

    def twall(x):
        return P["T_lo"] + P["T_lo_amp"] * cos(2 * pi * x / nx)

    def ob(z, y, x):
        return mask[z][y][x] != 0

    def nb(F, z, y, x, c, kind):
        """Neighbour value for the stencils; kind 's' (phi, C, f_s, p), 'T',
        'u' (a velocity component)."""
        xx, yy, zz = (x + c[0]) % nx, (y + c[1]) % ny, z + c[2]
        if 0 <= zz < nz:
            if ob(zz, yy, xx):
                if kind == "s":
                    return F[z][y][x]
                if kind == "u":
                    return -F[z][y][x]
            return F[zz][yy][xx]
        if zz < 0:
            m = F[-1 - zz][yy][xx]
            if kind == "T" and P["t_lo_dirichlet"]:
                return 2 * twall(xx) - m
        else:
            m = F[2 * nz - 1 - zz][yy][xx]
            if kind == "T" and P["t_hi_dirichlet"]:
                return 2 * P["T_hi"] - m
        return -m if kind == "u" else m

    def grad(F, z, y, x, kind):
        return [sum(W19[i] * C19[i][a] * nb(F, z, y, x, C19[i], kind) for i in range(1, 19)) / CS2
                for a in range(3)]

    def lap(F, z, y, x):
        return sum(2 * W19[i] * (nb(F, z, y, x, C19[i], "s") - F[z][y][x])
                   for i in range(1, 19)) / CS2

    grid = lambda: [[[mpf(0)] * nx for _ in range(ny)] for _ in range(nz)]
    D = grid()
    for (z, y, x) in nodes:
        if not ob(z, y, x):
            D[z][y][x] = (grad(state["ux"], z, y, x, "u")[0] + grad(state["uy"], z, y, x, "u")[1]
                          + grad(state["uz"], z, y, x, "u")[2])
    phi, T, C, fs, md, Q, E, rho, rc = (grid() for _ in range(9))
    for (z, y, x) in nodes:
        phi0 = sum(pops["f"][i][z][y][x] for i in range(7))
        E0 = sum(pops["h"][i][z][y][x] for i in range(7))
        Cs = sum(pops["l"][i][z][y][x] for i in range(7))
        if ob(z, y, x):
            Tn, _ = emap(P, E0, mpf(0))
            phi[z][y][x], C[z][y][x], T[z][y][x], E[z][y][x] = mpf(-1), mpf(0), Tn, E0
            rho[z][y][x] = P["rho_g"]
            rc[z][y][x] = P["rho_g"] * P["cp_g"]
            continue
        psi = min(max((1 + phi0) / 2, mpf(0)), mpf(1))
        ph = phi0 / (1 - D[z][y][x] / 2)
        T0, fs0 = emap(P, E0, psi)
        q = (prop(ph, fs0, P["rho_l"], P["rho_g"], P["rho_s"])
             * prop(ph, fs0, P["cp_l"], P["cp_g"], P["cp_s"]) * T0 * D[z][y][x])
        Ex = E0 + q / 2
        Tn, fsn = emap(P, Ex, psi)
        phi[z][y][x], T[z][y][x], fs[z][y][x], Q[z][y][x], E[z][y][x] = ph, Tn, fsn, q, Ex
        C[z][y][x] = Cs
        md[z][y][x] = ratio * (fsn - state["fs"][z][y][x])
        rho[z][y][x] = prop(ph, fsn, P["rho_l"], P["rho_g"], P["rho_s"])
        rc[z][y][x] = rho[z][y][x] * prop(ph, fsn, P["cp_l"], P["cp_g"], P["cp_s"])
    post = {k: [grid() for _ in range(len(pops[k]))] for k in pops}
    new_state = {k: grid() for k in state}
    alpha = 3 * sqrt(2) * eps / 4
    zero = [mpf(0)] * 3

    def heq(Ev, Tv, rcv, u):
        uu = dot(u, u)
        out = []
        for i in range(7):
            cu = dot(C7[i], u)
            if i == 0:
                out.append(Ev - P["rhoc_ref"] * Tv
                           + W7[0] * (P["rhoc_ref"] * Tv - rcv * Tv * uu / (2 * CS2)))
            else:
                out.append(W7[i] * (P["rhoc_ref"] * Tv
                                    + rcv * Tv * (cu / CS2 + (cu * cu - CS2 * uu) / (2 * CS2 ** 2))))
        return out

    def trt(z, y, x, he, src):
        for i in range(7):
            o = _opp(C7[i], C7)
            hi, ho = pops["h"][i][z][y][x], pops["h"][o][z][y][x]
            post["h"][i][z][y][x] = (hi - ((hi + ho) / 2 - (he[i] + he[o]) / 2) / tau_s
                                     - ((hi - ho) / 2 - (he[i] - he[o]) / 2) / tau_a
                                     + (1 - 1 / (2 * tau_s)) * W7[i] * src)

    for (z, y, x) in nodes:
        if ob(z, y, x):
            trt(z, y, x, heq(E[z][y][x], T[z][y][x], rc[z][y][x], zero), mpf(0))
            continue
        gp = grad(phi, z, y, x, "s")
        gT = grad(T, z, y, x, "T")
        gC = grad(C, z, y, x, "s")
        gf = grad(fs, z, y, x, "s")
        gP = grad(state["p"], z, y, x, "s")
        lp = lap(phi, z, y, x)
        gr = [(P["rho_l"] - P["rho_g"]) / 2 * gp[a] + (P["rho_s"] - P["rho_l"]) * gf[a]
              for a in range(3)]
        ng = sqrt(dot(gp, gp))
        den = max(ng, mpf("1e-6"))
        nv = [gp[a] / den for a in range(3)]
        ph = phi[z][y][x]
        mu = ph * (ph ** 2 - 1) / eps ** 2 - lp
        sig = (P["sigma0"] + P["sigma_T"] * (T[z][y][x] - P["T_ref"])
               + P["sigma_c"] * (C[z][y][x] - P["c_ref"]))
        gs = [P["sigma_T"] * gT[a] + P["sigma_c"] * gC[a] for a in range(3)]
        wst = (1 - fs[z][y][x]) if int(P["surface_tension_mode"]) == 0 else 1
        gsdp = dot(gs, gp)
        F = [wst * (alpha * sig * mu * gp[a] + alpha * (ng * ng * gs[a] - gsdp * gp[a]))
             + P["body_force"][a] for a in range(3)]
        g = [pops["g"][i][z][y][x] for i in range(19)]
        r = rho[z][y][x]
        us = [(sum(C19[i][a] * g[i] for i in range(19)) + F[a] / 2) / r for a in range(3)]
        fd = [-fs[z][y][x] * us[a] for a in range(3)]
        u = [us[a] + fd[a] / 2 for a in range(3)]
        S = r * md[z][y][x] + dot(u, gr)
        Ft = [F[a] - gP[a] + CS2 * gr[a] for a in range(3)]
        Ff = [F[a] + r * fd[a] for a in range(3)]
        G = []
        for i in range(19):
            c = C19[i]
            A = sum((u[a] * Ft[b] + Ft[a] * u[b]) * (c[a] * c[b] - (CS2 if a == b else 0))
                    for a in range(3) for b in range(3))
            G.append(W19[i] * (S + dot(c, Ff) / CS2 + A / (2 * CS2 ** 2)))
        uu = dot(u, u)
        s0 = W19[0] * (-uu / (2 * CS2))
        pn = CS2 / (1 - W19[0]) * (sum(g[1:]) + S / 2 + (tau_g - mpf(1) / 2) * G[0] + r * s0)
        for i in range(19):
            cu = dot(C19[i], u)
            si = W19[i] * (cu / CS2 + cu * cu / (2 * CS2 ** 2) - uu / (2 * CS2))
            geq = pn / CS2 * ((W19[i] - 1) if i == 0 else W19[i]) + r * si
            post["g"][i][z][y][x] = g[i] - (g[i] - geq) / tau_g + (1 - 1 / (2 * tau_g)) * G[i]
        B = [ph * u[a] - state["phi"][z][y][x] * state["u" + "xyz"[a]][z][y][x]
             + CS2 * nv[a] * (1 - ph * ph) * isq for a in range(3)]
        for i in range(7):
            c = C7[i]
            Fi = W7[i] * dot(c, B) / CS2 + W7[i] * ph * D[z][y][x]
            feq = W7[i] * ph * (1 + dot(c, u) / CS2)
            fi = pops["f"][i][z][y][x]
            post["f"][i][z][y][x] = fi - (fi - feq) / tau_f + (1 - 1 / (2 * tau_f)) * Fi
        trt(z, y, x, heq(E[z][y][x], T[z][y][x], rc[z][y][x], u), Q[z][y][x])
        f_s = fs[z][y][x]
        keff = 1 - f_s * (1 - P["k_p"])
        tau_l = (f_s * P["k_p"] * Ds + (1 - f_s) * Dl) / (CS2 * keff) + mpf(1) / 2
        Cc = C[z][y][x]
        R = [(1 - ph) * Cc * nv[a] * isq + (P["k_p"] - 1) * Cc * gf[a] / keff for a in range(3)]
        Lv = [Cc * u[a] - state["C"][z][y][x] * state["u" + "xyz"[a]][z][y][x] + CS2 * R[a]
              for a in range(3)]
        for i in range(7):
            c = C7[i]
            Li = W7[i] * dot(c, Lv) / CS2
            leq = W7[i] * Cc * (1 + dot(c, u) / CS2)
            li = pops["l"][i][z][y][x]
            post["l"][i][z][y][x] = li - (li - leq) / tau_l + (1 - 1 / (2 * tau_l)) * Li
        new_state["fs"][z][y][x] = f_s
        new_state["p"][z][y][x] = pn
        for a in range(3):
            new_state["u" + "xyz"[a]][z][y][x] = u[a]
        new_state["phi"][z][y][x] = ph
        new_state["C"][z][y][x] = Cc
    for (z, y, x) in nodes:
        if ob(z, y, x):
            new_state["phi"][z][y][x] = phi[z][y][x]
    # streaming: push each post-collision population along its link
    new = {k: [grid() for _ in range(len(pops[k]))] for k in pops}
    for k, lst in (("f", C7), ("g", C19), ("h", C7), ("l", C7)):
        for (z, y, x) in nodes:
            if k != "h" and ob(z, y, x):
                continue        # f, g, l are zero on an obstacle and never leave it
            for i, c in enumerate(lst):
                val = post[k][i][z][y][x]
                tx, ty, tz = (x + c[0]) % nx, (y + c[1]) % ny, z + c[2]
                o = _opp(c, lst)
                if 0 <= tz < nz:
                    if k != "h" and ob(tz, ty, tx):
                        new[k][o][z][y][x] = val      # bounced back by the obstacle
                    else:
                        new[k][i][tz][ty][tx] = val
                    continue
                if k == "h" and tz < 0 and P["t_lo_dirichlet"]:
                    val = -val + 2 * W7[o] * P["rhoc_ref"] * twall(x)
                elif k == "h" and tz >= nz and P["t_hi_dirichlet"]:
                    val = -val + 2 * W7[o] * P["rhoc_ref"] * P["T_hi"]
                new[k][o][z][y][x] = val
    return new, new_state
