"""FP64 PyTorch (CPU) version of the oracle step, for exact discrete gradients.

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline).  It computes the
same discrete map as lbf_oracle.c, written independently with whole-lattice
tensor operations, so that torch.autograd yields the exact gradient of a loss
of the final fields with respect to the per-node wettability cos(theta) and
the wall temperatures (through the initialisation and every step).  Its
forward map is checked against the C oracle to round-off.

State (the paper's notation): post-streaming f, g, h [9, ny, nx] and the
lagged fields f_s, Q = rho C_p T mdot, (phi u)_x, (phi u)_y, p, u_x, u_y of the
previous step.  Readings R1-R54 as in the C oracle.
"""

from __future__ import annotations

from typing import Dict, Tuple

import numpy as np
import torch

CX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
CY = [0, 0, 1, 0, -1, 1, 1, -1, -1]
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]
W = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
CS2 = 1.0 / 3.0
DT = torch.float64


def _col(v):
    return torch.tensor(v, dtype=DT).view(9, 1, 1)


class TorchLattice:
    """Geometry and index maps of one lattice (built once, no gradients)."""

    def __init__(self, case):
        self.case = case
        self.nx, self.ny = nx, ny = case.nx, case.ny
        self.m = case.mat
        m = self.m
        self.Eref = m.rho_ref * 2.0 * m.cp_s * m.cp_l / (m.cp_s + m.cp_l)
        self.w = _col(W)
        self.cx = _col(CX)
        self.cy = _col(CY)
        yy, xx = np.mgrid[0:ny, 0:nx]
        node = yy * nx + xx
        # stencil neighbours (wrap or mirror ghost), [9, ny*nx]
        nb = np.zeros((9, ny * nx), dtype=np.int64)
        for i in range(9):
            x2, y2 = xx + CX[i], yy + CY[i]
            x2 = np.where(x2 < 0, nx - 1 if case.periodic_x else 0, x2)
            x2 = np.where(x2 >= nx, 0 if case.periodic_x else nx - 1, x2)
            y2 = np.where(y2 < 0, ny - 1 if case.periodic_y else 0, y2)
            y2 = np.where(y2 >= ny, 0 if case.periodic_y else ny - 1, y2)
            nb[i] = (y2 * nx + x2).ravel()
        self.nb = torch.from_numpy(nb)
        # pull sources: plane*N + node of the population each node pulls
        N = nx * ny
        src = np.zeros((9, N), dtype=np.int64)
        wall = np.full((9, N), -1, dtype=np.int64)
        along = np.zeros((9, N), dtype=np.int64)
        for i in range(9):
            sx, sy = xx - CX[i], yy - CY[i]
            wl = np.full(sx.shape, -1)
            ylow, yhigh = sy < 0, sy >= ny
            if case.periodic_y:
                sy = np.mod(sy, ny)
            else:
                wl = np.where(ylow, 0, np.where(yhigh, 1, wl))
            xlow, xhigh = sx < 0, sx >= nx
            if case.periodic_x:
                sx = np.mod(sx, nx)
            else:
                wl = np.where((wl < 0) & xlow, 2, np.where((wl < 0) & xhigh, 3, wl))
            isw = wl >= 0
            own = node
            s = np.where(isw, OPP[i] * N + own, i * N + np.clip(sy, 0, ny - 1) * nx
                         + np.clip(sx, 0, nx - 1))
            src[i] = s.ravel()
            wall[i] = wl.ravel()
            along[i] = np.where(wl <= 1, xx, yy).ravel()
        self.src = torch.from_numpy(src.ravel())
        self.wall = torch.from_numpy(wall)
        self.along = torch.from_numpy(along)
        dirich = np.zeros((9, N), dtype=bool)
        for wv in range(4):
            if case.thermal_bc[wv]:
                dirich |= wall == wv
        self.dirich = torch.from_numpy(dirich)
        self.phi0 = torch.from_numpy(np.ascontiguousarray(case.phi0, dtype=np.float64))
        self.lap_phi0 = self.lap(self.phi0)

    # ---- stencils (isotropic D2Q9, wrap / mirror ghosts)
    def nbv(self, X):
        return X.reshape(-1)[self.nb].view(9, self.ny, self.nx)

    def grad(self, X):
        v = self.nbv(X)
        return (3.0 * (self.w * self.cx * v).sum(0), 3.0 * (self.w * self.cy * v).sum(0))

    def lap(self, X):
        v = self.nbv(X)
        return 6.0 * (self.w * (v - X)).sum(0)

    # ---- properties
    @staticmethod
    def zeta(s, C, zs, zl, zg):
        return s * zs + (1.0 - s) * (C * zl + (1.0 - C) * zg)

    def capacities(self, phi0, C, chi):
        m = self.m
        s_sol = torch.clamp(phi0 + chi, max=1.0)
        Kliq = self.zeta(phi0, C, m.rho_s, m.rho_l, m.rho_g) * self.zeta(phi0, C, m.cp_s, m.cp_l, m.cp_g)
        Ksol = self.zeta(s_sol, C, m.rho_s, m.rho_l, m.rho_g) * self.zeta(s_sol, C, m.cp_s, m.cp_l, m.cp_g)
        return Ksol, Kliq

    def hmap(self, rhoH, phi0, C, chi):
        m = self.m
        Ksol, Kliq = self.capacities(phi0, C, chi)
        Es = Ksol * m.T_m
        El = Kliq * m.T_m + chi * m.rho_l * m.latent
        sol = rhoH < Es
        liq = (~sol) & (rhoH > El)
        span = El - Es
        safe = torch.where(span > 0, span, torch.ones_like(span))
        fl_m = torch.where(span > 0, (rhoH - Es) / safe, torch.ones_like(span))
        fl = torch.where(sol, torch.zeros_like(rhoH), torch.where(liq, torch.ones_like(rhoH), fl_m))
        T = torch.where(sol, rhoH / Ksol,
                        torch.where(liq, m.T_m + (rhoH - El) / Kliq, torch.full_like(rhoH, m.T_m)))
        return T, fl, Ksol, Kliq

    def chem_pot(self, phi, lphi, cth, fs, lfs):
        m = self.m
        a, k = 3.0 * m.sigma / m.eps, 3.0 * m.eps * m.sigma / 8.0
        phi0 = self.phi0
        mu = a * phi * (phi * phi - 1.0) - k * lphi
        mu = mu + 3.0 * a * phi0 * phi0 * phi + a * cth * phi0 * (3 * phi * phi + phi0 * phi0 - 1.0) \
            - k * cth * self.lap_phi0
        mu = mu + 3.0 * a * fs * fs * phi + a * m.cos_psi * fs * (3 * phi * phi + fs * fs - 1.0) \
            - k * m.cos_psi * lfs
        return mu

    def liquid_weight(self, phihat):
        C = torch.clamp(0.5 * (1.0 - self.phi0 + phihat), 0.0, 1.0)
        Cp = torch.clamp((C - self.m.pcm_floor) / (1.0 - self.m.pcm_floor), 0.0, 1.0)
        return C, Cp

    @staticmethod
    def clamp_hi(v, lo, hi):
        # v < lo -> lo, else v > hi -> hi (the oracle's order)
        return torch.where(v < lo, lo, torch.where(v > hi, hi, v))

    # ---- initial state (u = 0, p = 0, equilibria, PCM liquid)
    def init_state(self, cth, phi=None, T0=None):
        m = self.m
        phi = torch.from_numpy(np.asarray(self.case.phi, dtype=np.float64)) if phi is None else phi
        T0 = torch.from_numpy(np.asarray(self.case.T, dtype=np.float64)) if T0 is None else T0
        zero = torch.zeros_like(phi)
        mu = self.chem_pot(phi, self.lap(phi), cth, zero, zero)
        C, Cp = self.liquid_weight(phi)
        chi = self.clamp_hi(Cp, torch.zeros_like(Cp), 1.0 - self.phi0)
        Ksol, Kliq = self.capacities(self.phi0, C, chi)
        rhoH = Kliq * (T0 - m.T_m) + Kliq * m.T_m + chi * m.rho_l * m.latent
        d0 = (torch.arange(9) == 0).to(DT).view(9, 1, 1)
        g = d0 * phi + (self.w - d0) * mu
        ET = self.Eref * T0
        h = d0 * (rhoH - ET) + self.w * ET
        f = torch.zeros((9,) + phi.shape, dtype=DT)
        lag = tuple(torch.zeros_like(phi) for _ in range(7))
        return f, g, h, lag

    # ---- one step
    def moments(self, g, h, lag):
        m = self.m
        fs_prev, Q_prev = lag[0], lag[1]
        phihat = g.sum(0)
        C, Cp = self.liquid_weight(phihat)
        chi = torch.maximum(Cp, fs_prev) if m.latch_fs else Cp
        chi = self.clamp_hi(chi, torch.zeros_like(chi), 1.0 - self.phi0)
        rhoH = h.sum(0) + 0.5 * Q_prev
        T, fl, Ksol, Kliq = self.hmap(rhoH, self.phi0, C, chi)
        fs = chi * (1.0 - fl)
        fstot = torch.clamp(self.phi0 + fs, max=1.0)
        mdot = (1.0 - m.rho_s / m.rho_l) * (fs - fs_prev)
        # div u of the phase-field source: mdot (R12) or the divergence of
        # the previous step's velocity (R54)
        if getattr(m, "phi_src_mdot", 0):
            divu = mdot
        else:
            divu = self.grad(lag[5])[0] + self.grad(lag[6])[1]
        phi = phihat / (1.0 - 0.5 * divu)
        rho = self.zeta(fstot, C, m.rho_s, m.rho_l, m.rho_g)
        return dict(phihat=phihat, C=C, chi=chi, rhoH=rhoH, T=T, fl=fl, fs=fs, fstot=fstot,
                    mdot=mdot, divu=divu, phi=phi, rho=rho, Ksol=Ksol, Kliq=Kliq)

    def step(self, state, cth, wallT):
        """wallT: tensor [4, max(nx, ny)] of wall temperatures."""
        m = self.m
        f, g, h, lag = state
        fs_prev, Q_prev, jx_prev, jy_prev, p_prev = lag[:5]
        M = self.moments(g, h, lag)
        phi, rho, C, fs, fstot, mdot, T = (M[k] for k in ("phi", "rho", "C", "fs", "fstot",
                                                            "mdot", "T"))
        mu_v = self.zeta(fstot, C, m.mu_s, m.mu_l, m.mu_g)
        lam = self.zeta(fstot, C, m.lam_s, m.lam_l, m.lam_g)
        cp = self.zeta(fstot, C, m.cp_s, m.cp_l, m.cp_g)
        tau_f = mu_v / rho / CS2 + 0.5
        tau_a = lam / self.Eref / CS2 + 0.5
        tau_s = 1.0 / (2.0 - 1.0 / tau_a)
        tau_g = m.mobility / CS2 + 0.5
        gphx, gphy = self.grad(phi)
        lphi = self.lap(phi)
        lfs = self.lap(fs)
        grx, gry = self.grad(rho)
        gpx, gpy = self.grad(p_prev)
        mu = self.chem_pot(phi, lphi, cth, fs, lfs)
        Fx, Fy = mu * gphx, mu * gphy
        mx, my = (self.cx * f).sum(0), (self.cy * f).sum(0)
        sum_nz = f[1:].sum(0)
        usx, usy = (mx + 0.5 * Fx) / rho, (my + 0.5 * Fy) / rho
        fdx, fdy = -fstot * usx, -fstot * usy
        ux, uy = usx + 0.5 * fdx, usy + 0.5 * fdy
        S = rho * mdot + ux * grx + uy * gry
        Ftx, Fty = Fx - gpx + CS2 * grx, Fy - gpy + CS2 * gry
        uu = ux * ux + uy * uy
        w0 = W[0]
        F0 = w0 * (S - (ux * Ftx + uy * Fty) / CS2)
        pr = CS2 / (1.0 - w0) * (sum_nz + 0.5 * S + (tau_f - 0.5) * F0 + rho * w0 * (-uu / (2 * CS2)))
        d0 = (torch.arange(9) == 0).to(DT).view(9, 1, 1)
        cu = self.cx * ux + self.cy * uy
        feq = pr / CS2 * (self.w - d0) + rho * self.w * (cu / CS2 + cu * cu / (2 * CS2 * CS2)
                                                           - uu / (2 * CS2))
        cF = self.cx * (Fx + rho * fdx) + self.cy * (Fy + rho * fdy)
        cFt = self.cx * Ftx + self.cy * Fty
        t2 = (2.0 * cu * cFt - CS2 * 2.0 * (ux * Ftx + uy * Fty)) / (2 * CS2 * CS2)
        Fi = self.w * (S + cF / CS2 + t2)
        fc = f - (f - feq) / tau_f + (1.0 - 0.5 / tau_f) * Fi
        jx, jy = phi * ux, phi * uy
        geq = d0 * phi + (self.w - d0) * mu + self.w * (self.cx * jx + self.cy * jy) / CS2
        Gi = self.w * (self.cx * (jx - jx_prev) + self.cy * (jy - jy_prev)) / CS2 \
            + self.w * phi * M["divu"]
        gc = g - (g - geq) / tau_g + (1.0 - 0.5 / tau_g) * Gi
        rhocp = rho * cp
        ET = self.Eref * T
        heq = d0 * (M["rhoH"] - ET + w0 * (ET - rhocp * T * uu / (2 * CS2))) + (1 - d0) * self.w * (
            ET + rhocp * T * (cu / CS2 + (cu * cu - CS2 * uu) / (2 * CS2 * CS2)))
        Q = rhocp * T * mdot
        tau_src = tau_a if m.h_src_tau_a else tau_s
        hb = h[OPP]
        eb = heq[OPP]
        ha, hs = 0.5 * (h - hb), 0.5 * (h + hb)
        ea, es = 0.5 * (heq - eb), 0.5 * (heq + eb)
        hc = h - (ha - ea) / tau_a - (hs - es) / tau_s + (1.0 - 0.5 / tau_src) * self.w * Q
        if self.case.substrate_fixed:
            Tw = self.case.T_substrate
            held = self.phi0 >= 0.5
            if Tw <= m.T_m:
                rH = M["Ksol"] * Tw
            else:
                rH = M["Kliq"] * (Tw - m.T_m) + M["Kliq"] * m.T_m + M["chi"] * m.rho_l * m.latent
            EW = self.Eref * Tw
            e = d0 * (rH - EW + w0 * EW) + (1 - d0) * self.w * EW
            hc = torch.where(held, e, hc)
        # streaming with bounce-back and anti-bounce-back
        N = self.nx * self.ny
        fn = fc.reshape(-1)[self.src].view(9, self.ny, self.nx)
        gn = gc.reshape(-1)[self.src].view(9, self.ny, self.nx)
        hn = hc.reshape(-1)[self.src].view(9, self.ny, self.nx)
        if self.dirich.any():
            wl = self.wall.clamp(min=0)
            twv = wallT[wl, self.along].view(9, self.ny, self.nx)
            d = self.dirich.view(9, self.ny, self.nx)
            hn = torch.where(d, -hn + 2.0 * self.w * self.Eref * twv, hn)
        lag_new = (fs, Q, jx, jy, pr, ux, uy)
        return (fn, gn, hn, lag_new)

    def fields(self, state):
        f, g, h, lag = state
        M = self.moments(g, h, lag)
        return M


def run(case, steps: int, cth=None, wallT=None, requires_grad: bool = False
        ) -> Tuple[Dict[str, torch.Tensor], torch.Tensor, torch.Tensor, "TorchLattice"]:
    """Initialise from the case and step; returns the final moments and the
    control tensors (cos theta per node, wall temperatures [4, max(nx, ny)])."""
    lat = TorchLattice(case)
    n = max(case.nx, case.ny)
    if cth is None:
        cth = torch.from_numpy(np.ascontiguousarray(case.cos_theta, dtype=np.float64))
    if wallT is None:
        wt = np.zeros((4, n))
        for w in range(4):
            p = case.wall_profile(w)
            wt[w, :len(p)] = p
        wallT = torch.from_numpy(wt)
    cth = cth.clone().requires_grad_(requires_grad)
    wallT = wallT.clone().requires_grad_(requires_grad)
    state = lat.init_state(cth)
    for _ in range(steps):
        state = lat.step(state, cth, wallT)
    return lat.fields(state), cth, wallT, lat


def run_checkpointed(case, steps: int, cth: torch.Tensor, wallT: torch.Tensor,
                     segment: int = 50) -> Tuple[Dict[str, torch.Tensor], "TorchLattice"]:
    """As run(), for long runs: the autograd graph is kept for one segment of
    steps at a time (torch.utils.checkpoint recomputes each segment in the
    backward pass), so memory grows with the number of segments, not steps.
    cth and wallT are used as given (leaf tensors with requires_grad, or
    expressions of them)."""
    from torch.utils.checkpoint import checkpoint
    lat = TorchLattice(case)
    state = lat.init_state(cth)
    flat = [state[0], state[1], state[2], *state[3]]

    def seg_fn(n, c, w, *xs):
        st = (xs[0], xs[1], xs[2], tuple(xs[3:10]))
        for _ in range(n):
            st = lat.step(st, c, w)
        return (st[0], st[1], st[2], *st[3])

    done = 0
    while done < steps:
        n = min(segment, steps - done)
        flat = list(checkpoint(seg_fn, n, cth, wallT, *flat, use_reentrant=True))
        done += n
    state = (flat[0], flat[1], flat[2], tuple(flat[3:10]))
    return lat.fields(state), lat
