"""MPS time stepper for eq. FP2 -- oracle (test infrastructure).

The scheme of the "Matrix product state algorithm" section: every vector of
eq. FP2 (the PDF f, the velocity components <U_i>, the mean compositions
<Phi_a>) is an MPS, every matrix (the CFD2 derivatives, diagonal
multiplications) an MPO, and the explicit Runge-Kutta update is carried out
in MPS arithmetic with the bond dimension of f limited to chi by singular
value truncation after every operator application and every stage
combination.

With the flow case's x-fields (a total diffusivity G(x) and an LMSE
frequency Omega_mix(x)), the constant-coefficient terms become
diag(G) D2p_i + diag(D1p_i G) D1p_i and diag(Omega) D1g diag(phi_a), and the
mean-field term uses the rounding of diag(Omega) <Phi_a>(x) with Omega = 1
in front.

Schedule of one RK4 step (RK2 is the Heun analogue):

    L(g)  = Round_chi( A(g) g ),   A(g) = A_fixed - Omega sum_a D1g^(phi_a) diag(m~_a(g))
    k1 = L(f); k2 = L(f + dt/2 k1); k3 = L(f + dt/2 k2)
    f+ = Round_chi( f + dt/6 k1 + dt/3 k2 + dt/3 k3 + dt/6 A(g4) g4 ),   g4 = f + dt k3

where the stage inputs f + c k are exact (block-diagonal) sums, the last
stage's product A(g4) g4 is never rounded by itself (its terms join the
final rounding: f is rounded once per step, each earlier slope once), m~_a(g) is
the raw mean composition of g rounded to chi_mean, and Round is the
randomized range finder followed by simultaneous SVD truncation
(``oracle.tt.round_sketch_two_sided``: the chain is orthogonalised from both
ends towards its middle site, then truncated simultaneously) with the
Gaussian sketches given as input.  This is ``rounding="sketch"``, the
schedule the GPU path runs.

``rounding="svd"`` is the paper's plain schedule instead: every operator
application A(g) g and every stage combination (the stage inputs
f + c k included) is formed explicitly and rounded by the textbook QR sweep
plus right-to-left truncated SVDs (``oracle.tt.round_ttsvd``); the mean
composition likewise.  It needs no random input and anchors the randomized
schedule: both approximate the same discrete solution, and the tests bound
the randomized step's distance to the full-grid solver by a small multiple
of this one's.

The operator MPOs are TT-SVDs of the dense 1-D matrices of ``oracle.dense``,
tensored over dimensions; nothing here is shared with the product path.

Pins: tests/test_oracle_stepper.py -- with chi >= 2^(N/2) (no truncation)
the stepper reproduces the full-grid solver of ``oracle.dense`` (itself
pinned to the paper's invariants and to closed forms) to 1e-12.
"""
from __future__ import annotations

import numpy as np

import workloads
from . import dense
from . import tt


class MPSStepper:
    def __init__(self, w, fields=None, rounding="sketch"):
        """fields: optional x-MPS cores of the flow case's variable
        coefficients, {"G": total diffusivity gamma + gamma_SGS (replaces the
        constant gamma), "Omega": LMSE frequency Omega_mix(x) (replaces the
        constant omega)}.  rounding: "sketch" (randomized two-sided range
        finder, the GPU path's schedule) or "svd" (the paper's plain
        schedule of explicit products rounded by QR + truncated SVDs)."""
        if rounding not in ("sketch", "svd"):
            raise ValueError(rounding)
        self.rounding = rounding
        self.w = w
        self.fields = dict(fields or {})
        self.order = workloads.site_order(w)
        self.N = len(self.order)
        self.nd = w.ndims
        self.M = w.M
        self.h = 1.0 / w.M
        self.n_phi = 2 * w.bits
        if w.ndims == 5 and w.ordering != "serial":
            raise ValueError("5-D problems use the serial ordering")
        M = self.M
        phi = dense.phi_nodes(M)
        self.ops = {
            "D1g": tt.operator_qtt(dense.d1_ghost(M)),
            "D2g": tt.operator_qtt(dense.d2_ghost(M)),
            "D1p": tt.operator_qtt(dense.d1_periodic(M)),
            "D2p": tt.operator_qtt(dense.d2_periodic(M)),
            "D1g_phi": tt.operator_qtt(dense.d1_ghost(M) @ np.diag(phi)),
            "phi": tt.operator_qtt(np.diag(phi)),
        }
        self.Z = workloads.sketch_cores(w)
        self.Zl = workloads.left_sketch_cores(w)
        self.ell = workloads.sketch_ranks(w)
        self.Zm = workloads.mean_sketch_cores(w)
        self.Zml = workloads.left_mean_sketch_cores(w)
        self.ell_m = workloads.mean_sketch_ranks(w)
        self.U = self._velocity() if w.ndims == 5 else None
        if self.fields and w.ndims != 5:
            raise ValueError("x-fields need a 5-D problem")
        self.dG = self._gradient(self.fields["G"]) if "G" in self.fields else None
        self.fixed = self._fixed_terms()
        self._weights = {}

    # ------------------------------------------------------------------ inputs
    def _x_order(self):
        return [(d - 2, b) for (d, b) in self.order if d >= 2]

    def _phi_order(self):
        return [(d, b) for (d, b) in self.order if d < 2]

    def _separable(self, terms, order, ndims):
        parts = []
        for c, vecs in terms:
            per = [None if v is None else tt.vector_qtt(v) for v in vecs]
            parts.append((c, tt.mps_product(per, order, ndims)))
        return tt.mps_sum(parts)

    def _velocity(self):
        out = []
        for comp in workloads.velocity_terms(self.w):
            x = self._separable(comp, self._x_order(), 3)
            x, _ = tt.round_det(x, self.w.vel_rank, self.w.rel_tol)
            out.append(x)
        return out

    def _gradient(self, G):
        """D1p_i G for i = 1, 2, 3 as exact x-MPSs (bond 3 times G's)."""
        out = []
        for i in range(3):
            per = [None] * 3
            per[i] = self.ops["D1p"]
            out.append(tt.mpo_apply(tt.mpo_product(per, self._x_order(), 3), G))
        return out

    def _x_diag(self, x):
        """diag(x) of an x-MPS, as an operator on the whole chain."""
        return tt.identity_mpo(self.n_phi) + tt.mpo_diag(x)

    def initial_state(self, with_info=False):
        f = self._separable(workloads.ic_terms(self.w), self.order, self.nd)
        f, info = tt.round_det(f, self.w.chi, self.w.rel_tol)
        return (f, info) if with_info else f

    # ---------------------------------------------------------------- operator
    def _mpo(self, per):
        return tt.mpo_product(per, self.order, self.nd)

    def _fixed_terms(self):
        w, o = self.w, self.ops
        nd = self.nd
        terms = []
        for a in (0, 1):
            per = [None] * nd
            per[a] = o["D1g_phi"]
            if "Omega" in self.fields:
                terms.append((1.0, tt.mpo_compose(self._x_diag(self.fields["Omega"]), self._mpo(per))))
            else:
                terms.append((w.omega, self._mpo(per)))
            per = [None] * nd
            per[a] = o["D2g"]
            terms.append((w.nu_phi, self._mpo(per)))
            if w.k_react != 0.0:
                per = [None] * nd
                per[a] = o["D1g_phi"]
                per[1 - a] = o["phi"]
                terms.append((w.k_react, self._mpo(per)))
        if nd == 5:
            for i in range(3):
                if "G" in self.fields:
                    per = [None] * nd
                    per[2 + i] = o["D2p"]
                    terms.append((1.0, tt.mpo_compose(self._x_diag(self.fields["G"]), self._mpo(per))))
                    per = [None] * nd
                    per[2 + i] = o["D1p"]
                    terms.append((1.0, tt.mpo_compose(self._x_diag(self.dG[i]), self._mpo(per))))
                elif w.gamma != 0.0:
                    per = [None] * nd
                    per[2 + i] = o["D2p"]
                    terms.append((w.gamma, self._mpo(per)))
                per = [None] * nd
                per[2 + i] = o["D1p"]
                D1 = self._mpo(per)
                diagU = tt.identity_mpo(self.n_phi) + tt.mpo_diag(self.U[i])
                terms.append((-1.0, tt.mpo_compose(diagU, D1)))
        return terms

    def _phi_weight(self, a):
        """Weight MPS over the phi sites for h^2 sum phi_a f (a = None: h^2 sum f)."""
        if a in self._weights:
            return self._weights[a]
        M = self.M
        vec = [np.full(M, self.h), np.full(M, self.h)]
        if a is not None:
            vec[a] = self.h * dense.phi_nodes(M)
        per = [tt.vector_qtt(v) for v in vec]
        W = tt.mps_product(per, self._phi_order(), 2)
        self._weights[a] = W
        return W

    def mean_field_raw(self, g, a):
        """<Phi_a>(x) of g: x-MPS (5-D) or scalar (2-D), unrounded."""
        W = self._phi_weight(a)
        v = np.ones((1, 1))
        for n in range(self.n_phi):
            v = np.einsum("wr,wsW,rsR->WR", v, W[n], g[n], optimize=True)
        if self.nd == 2:
            return float(v[0, 0])
        first = np.einsum("r,rsR->sR", v[0], g[self.n_phi])[None]
        return [first] + [G.copy() for G in g[self.n_phi + 1:]]

    def mean_field(self, g, a):
        """<Phi_a>(x) of g rounded to chi_mean; with an Omega field, the
        product Omega_mix(x) <Phi_a>(x) (the field enters the rounding as a
        diagonal operator)."""
        m = self.mean_field_raw(g, a)
        if self.nd == 2:
            return m, None
        W = tt.mpo_diag(self.fields["Omega"]) if "Omega" in self.fields else None
        if self.rounding == "svd":
            if W is not None:
                m = tt.mpo_apply(W, m)
            m, disc = tt.round_ttsvd(m, self.w.chi_mean, self.w.rel_tol)
            return m, {"discarded": disc}
        m, info = tt.round_sketch_two_sided([(1.0, W, m)], self.Zm, self.Zml,
                                            self.w.chi_mean, self.w.rel_tol)
        return m, info

    def operator_terms(self, g):
        w = self.w
        terms = list(self.fixed)
        for a in (0, 1):
            per = [None] * 2
            per[a] = self.ops["D1g"]
            phi_part = tt.mpo_product(per, self._phi_order(), 2)
            m, _ = self.mean_field(g, a)
            if self.nd == 2:
                terms.append((-w.omega * m, phi_part))
            else:
                om = 1.0 if "Omega" in self.fields else w.omega
                terms.append((-om, phi_part + tt.mpo_diag(m)))
        return terms

    def apply_exact(self, g):
        """A(g) g as an explicit (unrounded) MPS -- for small tests."""
        parts = [(c, tt.mpo_apply(W, g)) for c, W in self.operator_terms(g)]
        return tt.mps_sum(parts)

    def _round_explicit(self, x, chi):
        out, disc = tt.round_ttsvd(x, chi, self.w.rel_tol)
        return out, {"discarded": disc}

    def L(self, g):
        if self.rounding == "svd":
            return self._round_explicit(self.apply_exact(g), self.w.chi)
        terms = [(c, W, g) for c, W in self.operator_terms(g)]
        out, info = tt.round_sketch_two_sided(terms, self.Z, self.Zl, self.w.chi, self.w.rel_tol)
        return out, info

    def _combine(self, comb):
        """Round sum_j c_j x_j (comb = [(c_j, x_j)]) to chi."""
        if self.rounding == "svd":
            return self._round_explicit(tt.mps_sum(comb), self.w.chi)
        return tt.round_sketch_two_sided([(c, None, x) for c, x in comb], self.Z, self.Zl,
                                         self.w.chi, self.w.rel_tol)

    # -------------------------------------------------------------------- step
    def step(self, f):
        w = self.w
        dt = w.dt
        infos = []

        def L(g):
            out, info = self.L(g)
            infos.append(info)
            return out

        def stage_input(c, k):
            # exact block sum (sketch schedule) or rounded (plain schedule)
            g = tt.mps_sum([(1.0, f), (c, k)])
            if self.rounding == "svd":
                g, info = self._round_explicit(g, w.chi)
                infos.append(info)
            return g

        if w.integrator == "rk4":
            c_last, b = dt, [dt / 6, dt / 3, dt / 3, dt / 6]
            k1 = L(f)
            k2 = L(stage_input(0.5 * dt, k1))
            k3 = L(stage_input(0.5 * dt, k2))
            ks = [k1, k2, k3]
        elif w.integrator == "rk2":
            c_last, b = dt, [0.5 * dt, 0.5 * dt]
            ks = [L(f)]
        else:
            raise ValueError(w.integrator)
        g_last = stage_input(c_last, ks[-1])
        comb = [(1.0, f)] + [(bi, k) for bi, k in zip(b, ks)]
        if self.rounding == "svd":
            # the paper's plain schedule: the last product rounded, then the sum
            comb.append((b[-1], L(g_last)))
            fn, info = self._combine(comb)
        else:
            # the last stage's product A(g) g is not rounded by itself: its
            # terms, weighted by b_S, join the rounding of the combination
            terms = [(c, None, x) for c, x in comb]
            terms += [(b[-1] * c, W, g_last) for c, W in self.operator_terms(g_last)]
            fn, info = tt.round_sketch_two_sided(terms, self.Z, self.Zl, w.chi, w.rel_tol)
        infos.append(info)
        return fn, infos

    # ------------------------------------------------------------- observables
    def _weight_full(self, vecs):
        per = [tt.vector_qtt(v) for v in vecs]
        return tt.mps_product(per, self.order, self.nd)

    def observables(self, f):
        """Space-averaged statistics (eq. spaceAvg, eq. RACov, eq. SGSCov)."""
        M, h, nd = self.M, self.h, self.nd
        one = np.full(M, h)
        phi = h * dense.phi_nodes(M)
        xs = [one] * (nd - 2)
        mass = tt.inner(self._weight_full([one, one] + xs), f)
        m1 = tt.inner(self._weight_full([phi, one] + xs), f)
        m2 = tt.inner(self._weight_full([one, phi] + xs), f)
        m12 = tt.inner(self._weight_full([phi, dense.phi_nodes(M) * one] + xs), f)
        if nd == 2:
            avg_m1m2 = m1 * m2
        else:
            f1 = self.mean_field_raw(f, 0)
            f2 = self.mean_field_raw(f, 1)
            avg_m1m2 = h ** (nd - 2) * tt.inner(f1, f2)
        return {
            "mass": mass, "mean1": m1, "mean2": m2, "mean12": m12,
            "R12": avg_m1m2 - m1 * m2, "Y12": m12 - avg_m1m2,
            "product": mass - m1 - m2,
        }

    # ---------------------------------------------------------------- helpers
    def to_dense(self, f):
        return tt.sites_to_dense(tt.tt_full(f), self.order, self.w.bits, self.nd)

    def velocity_dense(self):
        """Densified velocity MPSs as (M, M, M) arrays (x1, x2, x3)."""
        if self.U is None:
            return None
        xo = self._x_order()
        return [tt.sites_to_dense(tt.tt_full(u), xo, self.w.bits, 3) for u in self.U]

    def dense_problem(self):
        w = self.w
        xo = self._x_order()
        fd = {k: tt.sites_to_dense(tt.tt_full(v), xo, w.bits, 3) for k, v in self.fields.items()}
        return dense.DenseProblem(w.ndims, w.M, w.omega, w.k_react, w.nu_phi,
                                  w.gamma if w.ndims == 5 else 0.0, self.velocity_dense(),
                                  G=fd.get("G"), Omega=fd.get("Omega"))
