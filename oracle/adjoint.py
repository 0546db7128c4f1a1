"""FP64 reverse-mode reference for the gradient of the summed sphere drag.

TEST INFRASTRUCTURE ONLY, like the rest of oracle/: nothing in the library
imports it.

The objective is J = sum_b F_b,x, the x-component of the force on every
sphere, summed over the spheres, at the last of n steps started from a fixed
state.  Its parameters are the body force F (3 values) and the sphere
velocities V (n_b x 3).  The spheres do not move (their positions are fixed;
V enters only through the moving-boundary term of Sec. 2.3, linear in V), the
box is periodic and has no walls.

The forward step of the oracle (streaming with the Bouzidi branches and the
moving-boundary term, momentum exchange, moments, the Smagorinsky tau*, BGK
with the Guo source; Sec. 2.2 and 2.3, readings as in lbm_oracle.c) is
restated with float64 torch tensors so that torch's reverse mode gives the
vector-Jacobian product of each step; the gradient then runs backwards over
the stored states, one step at a time.  The square root of Q = Pi:Pi has the
derivative 1/(2 sqrt(Q + EPS2)) (EPS2 = 1e-30), which is finite where Q = 0.

The restated step is pinned to the C oracle's step by test_oracle_adjoint.py,
and the gradient to central differences of the C oracle.
"""
import numpy as np
import torch

from . import Oracle, tables

EPS2 = 1e-30


class _Sqrt(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Q):
        ctx.save_for_backward(Q)
        return torch.sqrt(Q)

    @staticmethod
    def backward(ctx, g):
        (Q,) = ctx.saved_tensors
        return g / (2.0 * torch.sqrt(Q + EPS2))


def _min_image(d, L):
    return np.where(d > 0.5 * L, d - L, np.where(d < -0.5 * L, d + L, d))


class DragProblem:
    """Static geometry of an oracle run and its restated step."""

    def __init__(self, o: Oracle):
        if o.n_walls:
            raise ValueError("the drag gradient reference has no walls")
        self.nx, self.ny, self.nz = o.nx, o.ny, o.nz
        self.N = o.N
        tau0, C, rho0 = o.prm[:3]
        self.tau0, self.C, self.rho0 = float(tau0), float(C), float(rho0)
        self.halfway = bool(o.halfway)
        c, w, opp = tables()
        self.c = torch.tensor(c, dtype=torch.float64)
        self.ci = c
        self.w = torch.tensor(w, dtype=torch.float64)
        self.opp = opp
        B = o._bodies
        self.nb = B["n"]
        self.X = B["X"][: self.nb]
        self.R = B["R"][: self.nb]
        self.W = torch.tensor(B["W"][: self.nb], dtype=torch.float64)
        own = o.own
        self.fluid = torch.tensor(own < 0)
        self._links(own)

    def _links(self, own):
        """Every link from a fluid node x towards a sphere node x + c_k."""
        nx, ny, nz = self.nx, self.ny, self.nz
        n = np.arange(self.N)
        x, y, z = n % nx, (n // nx) % ny, n // (nx * ny)
        rows = []
        for k in range(1, 19):
            ck = self.ci[k]
            ns = ((x + ck[0]) % nx) + nx * (((y + ck[1]) % ny) + ny * ((z + ck[2]) % nz))
            sel = (own < 0) & (own[ns] >= 0)
            for xi in np.flatnonzero(sel):
                rows.append((xi, k, own[ns[xi]]))
        rows = np.array(rows, dtype=np.int64).reshape(-1, 3)
        xi, k, b = rows[:, 0], rows[:, 1], rows[:, 2]
        ck = self.ci[k].astype(np.float64)
        px, py, pz = xi % nx, (xi // nx) % ny, xi // (nx * ny)
        d = np.stack([_min_image(px - self.X[b, 0], nx), _min_image(py - self.X[b, 1], ny),
                      _min_image(pz - self.X[b, 2], nz)], 1)
        if self.halfway:
            q = np.full(len(xi), 0.5)
        else:
            a = (ck * ck).sum(1)
            bb = (d * ck).sum(1)
            cc = (d * d).sum(1) - self.R[b] ** 2
            q = np.clip((-bb - np.sqrt(np.maximum(bb * bb - a * cc, 0.0))) / a, 0.0, 1.0)
        xm = ((px - self.ci[k, 0]) % nx) + nx * (((py - self.ci[k, 1]) % ny) + ny * ((pz - self.ci[k, 2]) % nz))
        self.L = dict(x=torch.tensor(xi), k=torch.tensor(k), i=torch.tensor(self.opp[k].astype(np.int64)),
                      b=torch.tensor(b), q=torch.tensor(q), arm=torch.tensor(d + q[:, None] * ck),
                      xm=torch.tensor(xm), back_fluid=torch.tensor(own[xm] < 0))

    def step(self, P, F, V):
        """(P_n, force on every sphere) from P_{n-1}, the body force and V."""
        nx, ny, nz = self.nx, self.ny, self.nz
        c, w, L = self.c, self.w, self.L
        F = torch.as_tensor(F, dtype=torch.float64)
        V = torch.as_tensor(V, dtype=torch.float64)
        # pull streaming: f_i(x) = P(x - c_i)[i]
        f = torch.stack([torch.roll(P[i].view(nz, ny, nx), shifts=(int(self.ci[i, 2]), int(self.ci[i, 1]),
                                                                   int(self.ci[i, 0])), dims=(0, 1, 2)).reshape(-1)
                         for i in range(19)])
        # boundary links (Sec. 2.3)
        b, k, i, x, q = L["b"], L["k"], L["i"], L["x"], L["q"]
        uw = V[b] + torch.cross(self.W[b], L["arm"], dim=1)
        term = w[k] * self.rho0 * (c[i] * uw).sum(1)
        fk = P[k, x]
        lo = torch.where(L["back_fluid"], 2.0 * q * fk + (1.0 - 2.0 * q) * P[k, L["xm"]] + 6.0 * term,
                         fk + 6.0 * term)
        hi = fk / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * P[i, x] + 3.0 / q * term
        val = torch.where(q < 0.5, lo, hi)
        f = f.index_put((i, x), val)
        Fb = torch.zeros(self.nb, 3, dtype=torch.float64).index_add(0, b, (fk + val)[:, None] * c[k])
        # moments, equilibrium, Smagorinsky tau*, BGK + Guo (Sec. 2.2)
        rho = f.sum(0)
        u = (c.T @ f + 0.5 * F[:, None]) / rho
        cu = c @ u
        uu = (u * u).sum(0)
        feq = w[:, None] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)
        neq = f - feq
        Pi = torch.einsum("ia,ib,in->abn", c, c, neq)
        Q = (Pi * Pi).sum((0, 1))
        tau = 0.5 * (self.tau0 + torch.sqrt(self.tau0 ** 2 + 18.0 * np.sqrt(2.0) * self.C ** 2 * _Sqrt.apply(Q) / rho))
        cF = c @ F
        src = w[:, None] * (3.0 * (cF[:, None] - (F[:, None] * u).sum(0)) + 9.0 * cu * cF[:, None])
        Pn = f - neq / tau + (1.0 - 0.5 / tau) * src
        Pn = torch.where(self.fluid, Pn, P)  # solid nodes are never read back (spheres are fixed)
        return Pn, Fb

    def gradient(self, P0, F, V, nsteps):
        """J = sum_b F_b,x after nsteps steps from P0, and dJ/dF, dJ/dV."""
        F = torch.as_tensor(np.asarray(F, np.float64))
        V = torch.as_tensor(np.asarray(V, np.float64).reshape(self.nb, 3))
        states = [torch.as_tensor(np.asarray(P0, np.float64).reshape(19, self.N))]
        with torch.no_grad():
            for _ in range(nsteps - 1):
                states.append(self.step(states[-1], F, V)[0])
        gF = torch.zeros(3, dtype=torch.float64)
        gV = torch.zeros(self.nb, 3, dtype=torch.float64)
        lam = None
        J = None
        for n in range(nsteps, 0, -1):
            P = states[n - 1].clone().requires_grad_(True)
            Fr = F.clone().requires_grad_(True)
            Vr = V.clone().requires_grad_(True)
            Pn, Fb = self.step(P, Fr, Vr)
            if n == nsteps:
                J = Fb[:, 0].sum()
                out, gout = J, None
            else:
                out, gout = Pn, lam
            gP, gf, gv = torch.autograd.grad(out, (P, Fr, Vr), grad_outputs=gout, allow_unused=True)
            lam = gP
            if gf is not None:
                gF += gf
            if gv is not None:
                gV += gv
        return float(J.detach()), gF.numpy(), gV.numpy()
