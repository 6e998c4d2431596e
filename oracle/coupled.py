"""The IGA-ADS-CRVPINN coupled algorithm (oracle, test infrastructure).

Follows the IGA-ADS-CRVPINN algorithm section of the paper:
  1. inputs K, phi, sources, viscosities and S^0 as B-spline coefficients;
  2. pretrain the network on the robust loss with S^0;
  3. n = 1;
  4. L2-project the nodal network pressure into the B-spline space;
  5-6. explicit saturation update (eq. 6), repeated ten times with that pressure;
  7. retrain the network (100 Adam iterations) with the new saturation;
  8. stop or continue.

Readings:
  * step 8 returns to step 4, so every coupled step re-projects the pressure
    the network has just been trained to;
  * one coupled step of length dt runs the ten substeps with tau = dt / 10;
  * the nodal saturation used for alpha is the spline evaluated at the nodes;
  * Adam moments and step count persist across pretraining and all steps;
  * the network output is multiplied by the interior indicator (default) or,
    as an option, by the distance factor prod_a 4 x_a (1 - x_a): the paper
    only asks that the trial functions vanish on the boundary.
"""
from __future__ import annotations

import numpy as np

from . import ads, galerkin, mlp, pressure, wells as wells_mod


class Oracle:
    def __init__(self, dim, n_elem, degree, width, hidden, log_perm, porosity, wells,
                 theta0, s0_coefs=None, mu_w=1.0, mu_g=0.1, relperm_exp=2.0,
                 lr=1e-4, beta1=0.9, beta2=0.999, eps=1e-8, adam_iters=100,
                 substeps=10, well_radius=0.06, gravity=0.0, rho_w=0.0, rho_g=0.0,
                 boundary_factor=0):
        self.dim, self.n_elem, self.r = dim, n_elem, degree
        self.dims = mlp.layer_dims(dim, width, hidden)
        self.mu_w, self.mu_g, self.n_exp = mu_w, mu_g, relperm_exp
        self.gravity, self.rho_w, self.rho_g = gravity, rho_w, rho_g
        self.adam_iters, self.substeps = adam_iters, substeps
        self.log_perm = np.asarray(log_perm, dtype=np.float64).copy()
        self.perm = np.exp(self.log_perm)
        self.poro = np.asarray(porosity, dtype=np.float64)
        self.q_inj, self.q_prod = wells_mod.nodal_sources(wells, n_elem, dim, well_radius)
        self.q = self.q_inj + self.q_prod
        self.space = ads.Space(n_elem, degree, dim)
        nb = self.space.nb
        self.s = (np.zeros((nb,) * dim) if s0_coefs is None
                  else np.asarray(s0_coefs, dtype=np.float64).reshape((nb,) * dim).copy())
        self.theta = np.asarray(theta0, dtype=np.float64).copy()
        self.adam = mlp.Adam(self.theta.size, lr, beta1, beta2, eps)
        self.z = mlp.node_inputs(n_elem, dim)
        # trial-function factor: u = factor * NN (interior indicator, or the
        # distance form prod 4 x (1 - x) with boundary_factor = 1)
        if boundary_factor not in (0, 1):
            raise ValueError("boundary_factor must be 0 or 1")
        self.mask = (pressure.interior_mask(n_elem, dim) if boundary_factor == 0
                     else pressure.distance_factor(n_elem, dim))
        self.loss_history = []
        self.obs_d = self.obs_w = None
        self.refresh()

    # algorithm step 1 / after step 6: alpha from the current saturation
    def refresh(self):
        self.s_nodal = self.space.at_nodes(self.s)
        self.alpha = pressure.alpha_nodal(self.s_nodal, self.perm, self.mu_w,
                                          self.mu_g, self.n_exp)
        # right-hand side of the pressure system: wells minus the gravity
        # divergence (zero without gravity)
        self.q_eff = self.q - pressure.gravity_divergence(
            self.s_nodal, self.perm, self.mu_w, self.mu_g, self.n_exp, self.rho_w,
            self.rho_g, self.gravity)

    def u_nodal(self, theta=None):
        th = self.theta if theta is None else theta
        out = mlp.forward(th, self.dims, self.z)[-1]
        return self.mask * out.reshape(self.mask.shape)

    def set_observations(self, data, weights):
        """Nodal pressure observations d with weights w >= 0 (0: not
        observed); None clears them.  With observations the objective is
        LOSS + sum_p w_p (u_p - d_p)^2 (the data misfit of the inverse
        problem the paper names as future work)."""
        if data is None:
            self.obs_d = self.obs_w = None
            return
        self.obs_d = np.asarray(data, dtype=np.float64).reshape(self.mask.shape).copy()
        self.obs_w = np.asarray(weights, dtype=np.float64).reshape(self.mask.shape).copy()

    def loss_and_grad(self, theta=None):
        """Robust loss (plus the data misfit when observations are set) and
        its gradient with respect to the flat parameters."""
        th = self.theta if theta is None else theta
        acts = mlp.forward(th, self.dims, self.z)
        u = self.mask * acts[-1].reshape(self.mask.shape)
        res = pressure.residual(u, self.alpha, self.q_eff)
        q = pressure.gram_solve(res)
        lval = pressure.loss(res, q)
        gu = pressure.grad_u(q, self.alpha)
        if self.obs_w is not None:
            r = u - self.obs_d
            lval = lval + float(np.sum(self.obs_w * r * r))
            gu = gu + 2.0 * self.obs_w * r
        g = mlp.backward(th, self.dims, acts, (gu * self.mask).ravel())
        return lval, g

    def loss_grad_logperm(self, theta=None):
        """dLOSS/dlogK = dLOSS/dalpha * alpha (alpha is linear in K = e^logK),
        plus, with gravity, the part through the right-hand side: RES holds
        + h^d div_+(g F) with F linear in K, so the term is
        -2 gravity h^(d-1) F_m (q~_(m-e) - q~_m), q~ = q extended by zero."""
        th = self.theta if theta is None else theta
        u = self.u_nodal(th)
        res = pressure.residual(u, self.alpha, self.q_eff)
        q = pressure.gram_solve(res)
        g = pressure.grad_alpha(u, q) * self.alpha
        if self.gravity != 0.0:
            ne = self.n_elem
            h = 1.0 / ne
            f = pressure.buoyancy_flux(self.s_nodal, self.perm, self.mu_w, self.mu_g,
                                       self.n_exp, self.rho_w, self.rho_g)
            qt = np.zeros_like(u)
            qt[tuple(slice(1, ne) for _ in range(self.dim))] = q
            below = np.zeros_like(qt)
            below[1:] = qt[:-1]          # q~ at m - e_v
            g = g - 2.0 * self.gravity * h ** (self.dim - 1) * f * (below - qt)
        return g

    def set_log_perm(self, log_perm):
        self.log_perm = np.asarray(log_perm, dtype=np.float64).reshape(self.mask.shape).copy()
        self.perm = np.exp(self.log_perm)
        self.refresh()

    def invert(self, iters, lr_logk):
        """Joint Adam on the network parameters and the nodal log K, both at
        the gradient of the objective at the current (theta, log K): the
        parameters with the configured Adam, log K with a second Adam of rate
        lr_logk (same betas and eps) whose moments and step count start at
        zero with the first call.  K = exp(log K) and alpha follow each step."""
        if not hasattr(self, "lk_m"):
            self.lk_m = np.zeros_like(self.log_perm)
            self.lk_v = np.zeros_like(self.log_perm)
            self.lk_t = 0
        a = self.adam
        for _ in range(iters):
            lval, g = self.loss_and_grad()
            glk = self.loss_grad_logperm()
            self.loss_history.append(lval)
            self.theta = a.step(self.theta, g)
            self.lk_t += 1
            self.lk_m = a.b1 * self.lk_m + (1.0 - a.b1) * glk
            self.lk_v = a.b2 * self.lk_v + (1.0 - a.b2) * glk * glk
            mhat = self.lk_m / (1.0 - a.b1 ** self.lk_t)
            vhat = self.lk_v / (1.0 - a.b2 ** self.lk_t)
            self.set_log_perm(self.log_perm - lr_logk * mhat / (np.sqrt(vhat) + a.eps))

    def train(self, iters):
        for _ in range(iters):
            lval, g = self.loss_and_grad()
            self.loss_history.append(lval)
            self.theta = self.adam.step(self.theta, g)

    def pretrain(self, iters):
        self.train(iters)

    def project_pressure(self):
        return ads.project_nodal(self.space, self.u_nodal())

    def step(self, dt):
        p = self.project_pressure()
        tau = dt / self.substeps
        for _ in range(self.substeps):
            self.s = ads.saturation_substep(self.space, self.s, p, self.perm, self.poro,
                                            self.q_inj, self.q_prod, tau, self.mu_w,
                                            self.mu_g, self.n_exp, self.rho_g, self.gravity)
        self.refresh()
        self.train(self.adam_iters)

    # the paper's direct-solver algorithm (IGA-ADS with the Galerkin pressure
    # system, eq. 15-20, in place of CRVPINN)
    def galerkin_pressure(self):
        """Pressure coefficients of the Galerkin system for the current saturation."""
        return galerkin.pressure_solve(self.space, self.s, self.perm, self.q, self.mu_w,
                                       self.mu_g, self.n_exp, self.gravity, self.rho_w,
                                       self.rho_g)

    def step_galerkin(self, dt, p_coefs):
        """Substeps with the given pressure coefficients, refresh, and the
        Galerkin pressure of the new saturation (returned): one pass of the
        saturation update and pressure solve of that algorithm."""
        tau = dt / self.substeps
        for _ in range(self.substeps):
            self.s = ads.saturation_substep(self.space, self.s, p_coefs, self.perm, self.poro,
                                            self.q_inj, self.q_prod, tau, self.mu_w,
                                            self.mu_g, self.n_exp, self.rho_g, self.gravity)
        self.refresh()
        return self.galerkin_pressure()

    def fields(self):
        return self.u_nodal(), self.s.copy(), self.space.at_nodes(self.s)

    def direct_pressure(self):
        return pressure.direct_solve(self.alpha, self.q_eff)


def cfl_dt(orc: Oracle, cfl: float = 0.5) -> float:
    """Step length from a CFL number (the configurations state only "CFL 0.5"):
    dt = cfl * h_e * phi_min / (max_s lambda_g'(s) * max_p K_p |nabla_+ p0_p|),
    with p0 the direct solve of the current pressure system and
    max lambda_g' = n / mu_g for kr_g = s^n on [0, 1]."""
    p0 = orc.direct_pressure()
    g = pressure.grad_plus_norm(p0)
    ne = orc.n_elem
    kmax = np.max(orc.perm[tuple(slice(0, ne) for _ in range(orc.dim))] * g)
    dlam = orc.n_exp / orc.mu_g
    return float(cfl * (1.0 / ne) * orc.poro.min() / (dlam * kmax))
