"""Steady 1-D Boltzmann problem with diffuse walls (Sec. 5, Appendix B):
first-order upwind finite volumes in x, the spectral velocity grid, the
binary operator (O2) in the residual and the linearized operator about each
cell's local Maxwellian (Algorithm 1) in the modified Newton step.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Discrete problem (Appendix B, eq. (discrete_eq)), cells j = 1..Nx on
[x_L, x_R], velocities v_k, h_v = 2L/n:
    T[f]_j = v1+ (f_j - f_{j-1})/dx + v1- (f_{j+1} - f_j)/dx
    r(f)_j = T[f]_j - Q[f_j, f_j] / Kn
with ghost cells from the fully accommodating walls (eq. (maxwell_bc)):
    f_0      = rho_L E_L,  rho_L = -sum_k v1- f_1  / sum_k v1+ E_L
    f_{Nx+1} = rho_R E_R,  rho_R =  sum_k v1+ f_Nx / (-sum_k v1- E_R)
with E_W = exp(-|v - u_W|^2 / (2 theta_W)): the wall density that makes the
discrete mass flux through each wall exactly zero (reading R17; the printed
constants sqrt(2 pi / theta_W) and (2 pi theta_W)^(-3/2) are its continuum
limit, whose O(h_v^2) half-range quadrature error would leak mass; rho_R is
read from the last cell -- the printed formula names f(x_L), an evident slip).
Mass constraint (eq. (total_mass); reading R18): the collision terms are made
exactly mass-conserving -- Q with the fix Q^_0 = 0 of Sec. 2.3 and the
Jacobian projected, P L P -- so with zero-flux walls every Newton step and
every Krylov vector has zero mass and the mass of the initial guess is kept.
The discrete constraint dx h_v^3 sum_j sum_k f_jk = C is imposed on the
initial guess (eq. (initial) rescaled by C over its discrete mass) and again
on every Newton iterate (a rescaling that is the identity to rounding when the
linear solve keeps the mass).
Modified Newton (eq. (modified_Newton)): f <- f - g with
    T[g]_j - (P L_j P)[g_j] / Kn = r(f)_j,
L_j the linearized operator about the local Maxwellian of f_j.  The oracle
solves that linear system to a tight tolerance with scipy's matrix-free
GMRES from zero (relative 1e-10, absolute 1e-3 of the Newton tolerance) -- or, for tiny sizes, with the dense matrix.
Residual norm: sqrt(dx h_v^3 sum r^2).  Initial guess eq. (initial).
"""
import math

import numpy as np

from . import alg1, binary, fast_direct, grid, projection


class Problem:
    def __init__(self, n, L, omega, nx, kn, theta_l, theta_r, u_l=(0, 0, 0), u_r=(0, 0, 0), x_l=-0.5, x_r=0.5,
                 mass=1.0, sphere=None, R=None):
        self.n, self.L, self.nx, self.kn = n, L, nx, kn
        self.plan = fast_direct.make_plan(n, L, omega, R=R) if R else fast_direct.make_plan(n, L, omega)
        self.sphere = sphere
        self.x_l, self.x_r, self.mass = x_l, x_r, mass
        self.dx = (x_r - x_l) / nx
        self.xc = x_l + (np.arange(nx) + 0.5) * self.dx
        self.hv = 2.0 * L / n
        v = grid.velocities(n, L)
        self.V = np.stack(np.meshgrid(v, v, v, indexing="ij"), axis=0)   # [3, n, n, n]
        v1 = self.V[0]
        self.vp, self.vm = np.maximum(v1, 0.0), np.minimum(v1, 0.0)
        self.theta_l, self.theta_r = theta_l, theta_r
        self.ML = self._wall(u_l, theta_l)
        self.MR = self._wall(u_r, theta_r)

    def _wall(self, u, th):
        d2 = sum((self.V[d] - u[d]) ** 2 for d in range(3))
        return np.exp(-d2 / (2 * th))

    # ---- transport with wall ghosts (linear in f) ---------------------------
    def ghosts(self, f):
        rho_l = -np.sum(self.vm * f[0]) / np.sum(self.vp * self.ML)
        rho_r = -np.sum(self.vp * f[-1]) / np.sum(self.vm * self.MR)
        return rho_l * self.ML, rho_r * self.MR

    def transport(self, f):
        g0, g1 = self.ghosts(f)
        ext = np.concatenate([g0[None], f, g1[None]], axis=0)
        return (self.vp * (ext[1:-1] - ext[:-2]) + self.vm * (ext[2:] - ext[1:-1])) / self.dx

    # ---- collision terms -----------------------------------------------------
    def moments(self, f):
        """Density, velocity, temperature of each cell (discrete sums)."""
        h3 = self.hv ** 3
        out = np.empty((f.shape[0], 5))
        for j in range(f.shape[0]):
            rho = h3 * np.sum(f[j])
            u = [h3 * np.sum(self.V[d] * f[j]) / rho for d in range(3)]
            e = h3 * np.sum(sum((self.V[d] - u[d]) ** 2 for d in range(3)) * f[j]) / (3 * rho)
            out[j] = [rho, *u, e]
        return out

    def q(self, f):
        return np.stack([binary.q_binary(self.plan, self.sphere, f[j], f[j], fix=1) for j in range(f.shape[0])])

    def lcons(self, g, params):
        """P L P about each cell's local Maxwellian (params [nx, 5])."""
        phis = projection.invariants(self.n, self.L)
        out = np.empty_like(g)
        for j in range(g.shape[0]):
            Mj = fast_direct.maxwellian_fields(self.plan, params[j, 0], params[j, 1:4], params[j, 4])[0]
            x = projection.project(g[j], Mj, phis)
            y = alg1.apply_batch(self.plan, x[None], params[j:j + 1])[0]
            out[j] = projection.project(y, Mj, phis)
        return out

    def total_mass(self, f):
        return self.dx * self.hv ** 3 * np.sum(f)

    def residual(self, f):
        return self.transport(f) - self.q(f) / self.kn

    def norm(self, r):
        return math.sqrt(self.dx * self.hv ** 3 * np.sum(r * r))

    def initial(self):
        """eq. (initial): C/(x_R - x_L) times the unit Maxwellian at the
        linearly interpolated wall temperature, u = 0."""
        th = ((self.x_r - self.xc) * self.theta_l + (self.xc - self.x_l) * self.theta_r) / (self.x_r - self.x_l)
        d2 = sum(self.V[d] ** 2 for d in range(3))
        return np.stack([self.mass / (self.x_r - self.x_l) * (2 * math.pi * t) ** -1.5 * np.exp(-d2 / (2 * t))
                         for t in th])

    # ---- the inner solve's preconditioner ----------------------------------------
    def collision_frequency(self, params_c):
        """nu(v) = iDFT[Omega DFT[M]] (eq. (20)): the loss frequency of L about M."""
        M = fast_direct.maxwellian_fields(self.plan, params_c[0], params_c[1:4], params_c[4])[0]
        return grid.idft3(self.plan.Omega * grid.dft3(M)).real

    def sweep(self, y, f):
        """One source-iteration sweep (Sec. 5.2, eq. (source_iteration)) as a preconditioner about the
        local Maxwellians of f: z solves
            v1 (z_c - z_{c-1})/dx + nu+_c z_c/Kn = y_c   (v1 > 0)
            v1 (z_{c+1} - z_c)/dx + nu+_c z_c/Kn = y_c   (v1 <= 0)
        with nu+ = max(nu, 0), an empty ghost right of the last cell and the
        left wall ghost rho_L E_L taken from z's own first cell; then the total
        of z is removed along f: z <- z - (sum z / sum f) f."""
        params = self.moments(f)
        nu = np.stack([np.maximum(self.collision_frequency(p), 0.0) for p in params])
        a = np.abs(self.V[0]) / self.dx
        neg, pos = self.V[0] <= 0, self.V[0] > 0
        z = np.zeros_like(y)
        prev = np.zeros_like(y[0])
        for c in range(self.nx - 1, -1, -1):
            z[c] = np.where(neg, (y[c] + a * prev) / (a + nu[c] / self.kn), 0.0)
            prev = z[c]
        prev, _ = self.ghosts(z)
        for c in range(self.nx):
            z[c] = np.where(pos, (y[c] + a * prev) / (a + nu[c] / self.kn), z[c])
            prev = z[c]
        return z - np.sum(z) / np.sum(f) * f

    # ---- modified Newton -----------------------------------------------------
    def newton_matrix(self, params):
        """Dense matrix of g -> T[g] - L_j[g_j]/Kn (columns by unit vectors)."""
        n3 = self.n ** 3
        N = self.nx * n3
        A = np.empty((N, N))
        eye = np.eye(N).reshape(N, self.nx, self.n, self.n, self.n)
        for c in range(N):
            A[:, c] = self.transport(eye[c]).reshape(-1)
        for j in range(self.nx):
            cols = np.zeros((n3, self.nx, self.n, self.n, self.n))
            for c in range(n3):
                cols[c, j].reshape(-1)[c] = 1.0
            Lj = np.stack([self.lcons(cols[c], params)[j].reshape(-1) for c in range(n3)], axis=1)
            A[j * n3:(j + 1) * n3, j * n3:(j + 1) * n3] -= Lj / self.kn
        return A

    def newton_operator(self, params):
        """g -> T[g] - L_j[g_j]/Kn on flattened vectors."""
        shape = (self.nx, self.n, self.n, self.n)

        def mv(x):
            g = np.asarray(x, dtype=np.float64).reshape(shape)
            return (self.transport(g) - self.lcons(g, params) / self.kn).reshape(-1)
        return mv

    def newton_step(self, f, r, dense=False, atol=0.0):
        """g with T[g] - P L P[g]/Kn = r about the local Maxwellians of f;
        GMRES stops at |residual| <= max(1e-10 |r|, atol)."""
        params = self.moments(f)
        if dense:
            return np.linalg.solve(self.newton_matrix(params), r.reshape(-1)).reshape(f.shape)
        import scipy.sparse.linalg as sla
        N = r.size
        op = sla.LinearOperator((N, N), matvec=self.newton_operator(params), dtype=np.float64)
        g, info = sla.gmres(op, r.reshape(-1), rtol=1e-10, atol=atol, restart=200, maxiter=20)
        if info != 0:
            raise RuntimeError(f"oracle GMRES did not converge ({info})")
        return g.reshape(f.shape)

    def constrain(self, f):
        """Rescales f to the discrete total mass C."""
        return f * (self.mass / self.total_mass(f))

    def solve(self, f=None, tol=1e-5, max_newton=20, dense=False):
        """Modified Newton iteration with (near-)exact linear solves.
        Returns (f, residual norms [one per evaluation])."""
        f = self.constrain(self.initial() if f is None else np.array(f, dtype=np.float64))
        hist = []
        for _ in range(max_newton + 1):
            r = self.residual(f)
            hist.append(self.norm(r))
            if hist[-1] < tol:
                break
            f = self.constrain(f - self.newton_step(f, r, dense, atol=1e-3 * tol))
        return f, hist
