"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test checks the oracle against something other than itself: closed forms, a textbook
routine, a special case that reduces to a 1D problem with an exact solution, invariants the
method has, or the paper's printed convergence orders.
"""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
from paper_2006_14602_amd import workloads as W

UNIT2 = ((0.0, 0.0), (1.0, 1.0))


def grid2(n, lo=(0.0, 0.0), hi=(1.0, 1.0)):
    return O.GridSpec((n, n), lo, hi)


# --- P10: theta = int rho (Sec. 2, normalisation before eq. edp) -----------------------------

def test_theta_ring_close_to_disk_form():
    # the sech^2 ring lies inside the unit square up to a tail of ~1e-8: the integral over the
    # inscribed disk of radius 1/2 is (pi/k)[tanh(k(1/4 - r0^2)) + tanh(k r0^2)]
    mon = W.ring_monitor()
    th = O.theta_quadrature(mon, *UNIT2)
    disk = 1.0 + 10.0 * (math.pi / 50.0) * (math.tanh(50.0 * (0.25 - 1.0 / 16.0)) + math.tanh(50.0 / 16.0))
    assert 0.0 < th - disk < 2e-8
    # the corner tail is what separates them; integrate it from the radial profile outside r=1/2
    assert abs(th - 2.2542158532) < 1e-9


def test_theta_sine_inner_integral_closed_form():
    # int_0^1 sech^2(k(y - 1/2 - s)) dy = [tanh(k(1/2 - s)) + tanh(k(1/2 + s))] / k
    mon = W.sine_monitor()
    inner = lambda x: (math.tanh(40 * (0.5 - 0.25 * math.sin(2 * math.pi * x)))
                       + math.tanh(40 * (0.5 + 0.25 * math.sin(2 * math.pi * x)))) / 40.0
    ref = 1.0 + 20.0 * scipy.integrate.quad(inner, 0, 1, epsabs=1e-15, epsrel=1e-15, limit=400)[0]
    assert abs(O.theta_quadrature(mon, *UNIT2) - ref) < 1e-12
    assert abs(ref - 1.99999999963) < 1e-10


@pytest.mark.parametrize("d", [2, 3])
def test_theta_gauss_erf_vs_quadrature(d):
    rng = np.random.default_rng(7)
    mon = {"kind": "gauss_sum", "bamp": [12.0, 25.0], "bw": [0.05, 0.12],
           "bc": [list(rng.uniform(0, 1, d)), list(rng.uniform(0, 1, d))]}
    lo, hi = (0.0,) * d, (1.0,) * d
    assert abs(O.theta_closed_form(mon, lo, hi) - O.theta_quadrature(mon, lo, hi, panels=48 if d == 3 else 128)) < 1e-11


def test_theta_separable_closed_form_vs_quadrature():
    mon = W.separable_monitor((8.0, 5.0), (20.0, 15.0), (0.4, 0.6))
    assert abs(O.theta_closed_form(mon, *UNIT2) - O.theta_quadrature(mon, *UNIT2)) < 1e-12


# --- discrete operators against analytic derivatives (second order, Sec. 3) ------------------

@pytest.mark.parametrize("d", [2, 3])
def test_fd_hessian_second_order_with_ghosts(d):
    # phi = eps prod_k cos(m_k pi xi_k) satisfies the homogeneous Neumann condition, so
    # Psi = |xi|^2/2 + phi satisfies eq. nbd exactly; the FD gradient and Hessian (including the
    # mixed terms and the corner ghosts) must converge at second order to the analytic ones.
    eps = 0.01
    m = (1, 2, 1)[:d]
    errs = []
    for n in ((17, 33) if d == 3 else (33, 65)):
        g = O.GridSpec((n,) * d, (0.0,) * d, (1.0,) * d)
        box = g.whole_box()
        X = box.coords()
        c = [np.cos(m[k] * np.pi * X[..., k]) for k in range(d)]
        s = [np.sin(m[k] * np.pi * X[..., k]) for k in range(d)]
        prod = lambda arrs: np.prod(np.stack(arrs), axis=0)
        psi = 0.5 * np.sum(X * X, axis=-1) + eps * prod(c)
        grad, hess = O.derivatives(psi, box)
        e = 0.0
        for k in range(d):
            gk = X[..., k] - eps * m[k] * np.pi * prod([s[j] if j == k else c[j] for j in range(d)])
            e = max(e, np.max(np.abs(grad[k] - gk)))
            for l in range(d):
                if l == k:
                    hk = 1.0 - eps * (m[k] * np.pi) ** 2 * prod(c)
                else:
                    hk = eps * m[k] * m[l] * np.pi ** 2 * prod([s[j] if j in (k, l) else c[j] for j in range(d)])
                e = max(e, np.max(np.abs(hess[k][l] - hk)))
        errs.append(e)
    order = math.log2(errs[0] / errs[1])
    assert 1.8 < order < 2.3, (errs, order)


def test_F_constant_monitor_is_log_det():
    # rho = 1, theta = 1, |Omega_c| = 1: F = log det D^2_h Psi exactly
    g = grid2(17)
    box = g.whole_box()
    X = box.coords()
    psi = 0.5 * np.sum(X * X, -1) + 0.02 * np.cos(np.pi * X[..., 0]) * np.cos(np.pi * X[..., 1])
    F = O.rhs_F(psi, box, W.const_monitor(), 1.0, 1.0)
    _, hess = O.derivatives(psi, box)
    np.testing.assert_array_equal(F, np.log(hess[0][0] * hess[1][1] - hess[0][1] ** 2))


# --- P6: the DCT-I preconditioner is the sparse direct solve of (I - gamma L_h) ---------------

@pytest.mark.parametrize("shape", [(9, 12), (5, 7, 6)])
def test_precondition_equals_sparse_solve(shape):
    rng = np.random.default_rng(1)
    h = tuple(1.0 / (n - 1) for n in shape)
    gam = 0.37
    F = rng.standard_normal(shape)
    L = None
    for k, n in enumerate(shape):
        term = sp.identity(1)
        for j, m in enumerate(shape):
            term = sp.kron(term, O.assemble_neumann_laplacian_1d(m, h[j]) if j == k else sp.identity(m))
        L = term if L is None else L + term
    A = (sp.identity(F.size) - gam * L).tocsc()
    ref = spla.spsolve(A, F.ravel()).reshape(shape)
    assert np.max(np.abs(O.precondition(F, h, gam) - ref)) < 1e-12 * np.max(np.abs(ref)) * 10


# --- P1: rho = 1 keeps Psi = |xi|^2/2 steady, identity mesh (Sec. 2) --------------------------

def test_constant_monitor_identity_mesh():
    g = grid2(33)
    r = O.solve_single(g, W.const_monitor(), 1e-3, 1.0, 30)
    X = np.moveaxis(g.whole_box().coords(), -1, 0)
    assert np.max(np.abs(r.mesh - X)) <= 1e-12
    assert np.max(np.abs(r.psi - 0.5 * np.sum(X * X, 0))) <= 1e-12


# --- P2: separable monitor -> sum of 1D iterates; steady 1D = exact equidistribution ---------

def test_separable_monitor_reduces_to_1d_iterates():
    A, K, C = (8.0, 5.0), (20.0, 15.0), (0.4, 0.6)
    g = O.GridSpec((33, 41), (0.0, 0.0), (1.0, 1.0))
    r2 = O.solve_single(g, W.separable_monitor(A, K, C), 1e-3, 1.0, 40)
    ones = []
    for ax in range(2):
        g1 = O.GridSpec((g.n[ax],), (0.0,), (1.0,))
        ones.append(O.solve_single(g1, W.separable_monitor((A[ax],), (K[ax],), (C[ax],)), 1e-3, 1.0, 40))
    assert np.max(np.abs(r2.psi - (ones[0].psi[:, None] + ones[1].psi[None, :]))) < 1e-12
    assert np.max(np.abs(r2.mesh[0] - ones[0].mesh[0][:, None])) < 1e-12
    assert np.max(np.abs(r2.mesh[1] - ones[1].mesh[0][None, :])) < 1e-12


def test_1d_steady_state_matches_exact_equidistribution_second_order():
    A, K, C = 8.0, 20.0, 0.4
    errs = []
    for n in (65, 129, 257):
        g1 = O.GridSpec((n,), (0.0,), (1.0,))
        r = O.solve_single(g1, W.separable_monitor((A,), (K,), (C,)), 0.05, 1.0, 2500)
        X = O.equidistribution_exact_sech2(np.linspace(0, 1, n), 0.0, 1.0, A, K, C)
        errs.append(np.max(np.abs(r.mesh[0] - X)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.85 < o < 2.15 for o in orders), (errs, orders)
    assert errs[-1] < 5e-5


# --- P3 / P4: exact DD identities --------------------------------------------------------------

@pytest.mark.parametrize("ov", [2, 4, 7])
def test_forward_euler_dd_equals_single_domain_exactly(ov):
    # gamma = 0, overlap >= 2 cells, time-n transmission: every subdomain reproduces the global
    # iterate on its live nodes (locality of the stencil), bit for bit.
    g = grid2(33)
    mon = W.ring_monitor()
    a = O.solve_single(g, mon, 1e-4, 0.0, 25)
    b = O.solve_dd(g, (2, 3), (ov, ov), mon, 1e-4, 0.0, 25)
    np.testing.assert_array_equal(a.mesh, b.mesh)
    np.testing.assert_array_equal(a.psi, b.psi)


def test_single_part_dd_equals_single_domain():
    g = grid2(33)
    mon = W.ring_monitor()
    a = O.solve_single(g, mon, 1e-3, 1.0, 20)
    b = O.solve_dd(g, (1, 1), (4, 4), mon, 1e-3, 1.0, 20)
    np.testing.assert_array_equal(a.mesh, b.mesh)


def test_partition_matches_worked_split():
    # 513 nodes, 4 parts, overlap 8 cells -> [0,132], [124,260], [252,388], [380,512]
    cores, ranges = O.partition_axis(512, 4, 8)
    assert cores == [0, 128, 256, 384, 512]
    assert ranges == [(0, 132), (124, 260), (252, 388), (380, 512)]
    assert O.partition_axis(128, 2, 6)[1] == [(0, 67), (61, 128)]
    own = O.owner_axis(np.array([0, 127, 128, 511, 512]), cores)
    assert list(own) == [0, 0, 1, 3, 3]


# --- P5: DD - single domain shrinks as the overlap grows (Sec. 4.4, overlap study) -----------

@pytest.mark.slow
def test_dd_error_falls_with_overlap():
    g = grid2(129)
    mon = W.ring_monitor()
    gam = 4.0 / 128 ** 2
    dt = 0.2 * gam
    steps = 205
    sd = O.solve_single(g, mon, dt, gam, steps)
    errs = [float(np.max(np.abs(O.solve_dd(g, (4, 4), (ov, ov), mon, dt, gam, steps).mesh - sd.mesh)))
            for ov in (4, 8, 16)]
    assert errs[0] > errs[1] > errs[2] > 0
    assert errs[0] / errs[2] > 3.0
    assert errs[0] < 3e-3


# --- P13: the DD fixed point is the whole-domain discrete steady state (Sec. 3, Sec. 4.4) ---------

@pytest.mark.parametrize("mode", ["parallel", "alternating"])
def test_dd_fixed_point_is_single_domain_steady_state(mode):
    # The discrete steady state of the whole-domain scheme has F equal to a constant c (the discrete
    # integral of rho det differs from theta by O(h^2)), and Psi then drifts by dt*c per step. With
    # theta scaled by exp(c) the steady state has F = 0 and no drift. A converged DD solve must then
    # satisfy the whole-domain equation F = 0 at every node of the glued Psi, and its mesh must be
    # the whole-domain steady mesh: the artificial-face values, the preconditioner's Neumann faces
    # and the F := 0 rows leave no trace in the fixed point.
    g = grid2(33)
    mon = W.ring_monitor(amp=5.0, k=10.0)
    box = g.whole_box()
    th = O.theta(mon, g.lo, g.hi)
    sd0 = O.solve_single(g, mon, 0.05, 1.0, 4000, tol=1e-14)
    c = float(np.mean(O.rhs_F(sd0.psi, box, mon, th, g.vol)))
    assert abs(c) > 1e-3     # the drift is real, so the rescaling below is not a no-op
    th0 = th * math.exp(c)
    sd = O.solve_single(g, mon, 0.05, 1.0, 4000, tol=1e-15, theta_val=th0)
    assert np.abs(O.rhs_F(sd.psi, box, mon, th0, g.vol)).max() < 1e-10
    gam = 4.0 / 32 ** 2
    dt = 0.2 * gam
    dd = O.solve_dd(g, (2, 2), (4, 4), mon, dt, gam, 20000, tol=1e-12, mode=mode, theta_val=th0)
    assert dd.res_hist[-1] <= 1e-12 and dd.steps < 20000
    F = O.rhs_F(dd.psi, box, mon, th0, g.vol)
    assert np.abs(F).max() < 1e-7
    assert np.max(np.abs(dd.mesh - sd.mesh)) < 1e-8
    # With the unscaled theta the DD iteration also stalls into a uniform drift, but its stationary
    # state is not the whole-domain one: F then varies near the artificial faces.
    dd_drift = O.solve_dd(g, (2, 2), (4, 4), mon, dt, gam, 1500, mode=mode, theta_val=th)
    F1 = O.rhs_F(dd_drift.psi, box, mon, th, g.vol)
    assert F1.max() - F1.min() > 1e-4


# --- P7 / P8 / P9: boundary, symmetry, positivity ---------------------------------------------

def test_ring_mesh_boundary_symmetry_positivity():
    g = grid2(65)
    r = O.solve_single(g, W.ring_monitor(), 1e-3, 1.0, 200)
    x, y = r.mesh
    # P7: nodes stay on the faces they started on (eq. nbd; eqs. adapt_mesh_bc1/2)
    assert np.max(np.abs(x[0, :] - 0.0)) < 1e-13 and np.max(np.abs(x[-1, :] - 1.0)) < 1e-13
    assert np.max(np.abs(y[:, 0] - 0.0)) < 1e-13 and np.max(np.abs(y[:, -1] - 1.0)) < 1e-13
    # P8: the ring is invariant under x <-> 1 - x and under the axis swap
    assert np.max(np.abs(x - (1.0 - x[::-1, :]))) < 1e-12
    assert np.max(np.abs(x - y.T)) < 1e-12
    # P9: convex potential, unfolded mesh (Sec. 2)
    assert r.min_det > 0 and r.min_cell > 0
    # the mesh has moved (the monitor is not trivial)
    assert np.max(np.abs(x - np.linspace(0, 1, 65)[:, None])) > 1e-2


def test_min_cell_measure_identity_and_fold():
    g = O.GridSpec((5, 6, 4), (0.0,) * 3, (1.0,) * 3)
    X = np.moveaxis(g.whole_box().coords(), -1, 0)
    assert abs(O.min_cell_measure(X) - np.prod(g.h)) < 1e-15
    Y = X.copy()
    Y[0, 2, 3, 1] += 0.6   # push a node past its neighbour: folds cells
    assert O.min_cell_measure(Y) < 0
    g2 = grid2(5)
    X2 = np.moveaxis(g2.whole_box().coords(), -1, 0)
    assert abs(O.min_cell_measure(X2) - 1.0 / 16) < 1e-15


def test_tangling_raises():
    g = grid2(65)
    with pytest.raises(O.TangledError):
        O.solve_single(g, W.ring_monitor(), 10.0 / 64 ** 2, 0.0, 100)


# --- P11: first order in pseudo time with forward Euler (Sec. 4.4, slopes near 1) -------------

@pytest.mark.slow
def test_forward_euler_first_order_in_time():
    mon = W.ring_monitor()
    n = 33
    h = 1.0 / (n - 1)
    g = grid2(n)
    ref = O.solve_single(g, mon, 0.0015 * h * h, 0.0, 16000)
    errs = []
    for c, st in ((0.015, 1600), (0.03, 800), (0.06, 400), (0.12, 200)):
        errs.append(O.rel_errors(ref.psi, O.solve_dd(g, (2, 2), (4, 4), mon, c * h * h, 0.0, st).psi, g.h))
    x = np.log([0.015, 0.03, 0.06, 0.12])
    for p in (1, 2, "inf"):
        slope = np.polyfit(x, np.log([e[p] for e in errs]), 1)[0]
        assert abs(slope - 1.0) < 0.15, (p, slope)


# --- P12: quality measure close to one (Sec. 4.5) ---------------------------------------------

def test_quality_measure_near_one():
    g = grid2(41)
    mon = W.ring_monitor()
    r = O.solve_single(g, mon, 0.05, 1.0, 1500)
    q = O.quality(r.psi, g, mon)
    assert abs(q["E2"] - 1.0) < 0.05
    assert 1.0 < q["Emax"] < 2.0


# --- residual definition (eq. dd_stop_criterion) -----------------------------------------------

def test_residual_is_trapezoid_norm_of_update():
    g = grid2(17)
    box = g.whole_box()
    mon = W.ring_monitor()
    psi0 = O.initial_psi(box)
    th = O.theta(mon, g.lo, g.hi)
    psi1, res = O.step_box(psi0, box, mon, th, 1.0, 1e-3, 1.0)
    diff = psi1 - psi0
    w = np.ones(g.n)
    w[0, :] *= 0.5
    w[-1, :] *= 0.5
    w[:, 0] *= 0.5
    w[:, -1] *= 0.5
    assert abs(res - math.sqrt(np.sum(w * diff ** 2) * g.h[0] * g.h[1])) < 1e-15


def test_transmission_sources_are_live_nodes():
    # every artificial node's source lies strictly inside its owner (checked while building)
    for parts, ov in (((4, 4), (8, 8)), ((3, 2), (2, 2)), ((2, 2, 2), (6, 6, 6))):
        d = len(parts)
        n = (33,) * d if d == 3 else (65, 49)
        dec = O.Decomposition(O.GridSpec(n, (0.0,) * d, (1.0,) * d), parts, ov)
        total_art = sum(int(s.box.artificial_mask().sum()) for s in dec.subs)
        total_listed = sum(len(dst) for lists in dec.trans for _, dst, _ in lists)
        assert total_art == total_listed


# --- Alternating DD (Algorithm 1): subdomains updated in turn, each reading the latest values --

def _boxes_and_owner(n, parts, ov):
    """Node ranges per axis, subdomain boxes (block order) and the global owner array, from the
    partition rule alone (pinned above by the worked split)."""
    d = len(n)
    axes = [O.partition_axis(n[k] - 1, parts[k], ov[k]) for k in range(d)]
    boxes = []
    for idx in np.ndindex(*parts):
        boxes.append(tuple(axes[k][1][idx[k]] for k in range(d)))
    own_axes = [O.owner_axis(np.arange(n[k]), axes[k][0]) for k in range(d)]
    own = np.ravel_multi_index(np.meshgrid(*own_axes, indexing="ij"), parts)
    return boxes, own


def _masks(n, box):
    """Global masks of a box's nodes and of its artificial (inner-face) nodes."""
    d = len(n)
    inside = np.ones(n, dtype=bool)
    art = np.zeros(n, dtype=bool)
    for k in range(d):
        idx = np.arange(n[k])
        lo, hi = box[k]
        shape = [1] * d
        shape[k] = -1
        inside &= ((idx >= lo) & (idx <= hi)).reshape(shape)
        face = np.zeros(n[k], dtype=bool)
        if lo > 0:
            face[lo] = True
        if hi < n[k] - 1:
            face[hi] = True
        art |= face.reshape(shape)
    art &= inside
    return inside, art


def _alternating_by_whole_domain_steps(g, parts, ov, mon, dt, steps, order):
    """Forward-Euler alternating DD written with whole-domain steps: every subdomain keeps a
    whole-grid field that is valid on its box.  Its turn: artificial nodes <- owners' latest
    values; one whole-domain Euler step of (other nodes from their owners, own box from its own
    field); keep the result on the box's non-artificial nodes.  The Euler stencil of a node
    that is not artificial stays inside the box, so this is the subdomain step exactly."""
    n = g.n
    boxes, own = _boxes_and_owner(n, parts, ov)
    th = O.theta(mon, g.lo, g.hi)
    psi0 = O.initial_psi(g.whole_box())
    fields = [psi0.copy() for _ in boxes]
    masks = [_masks(n, b) for b in boxes]

    def glued():
        out = np.empty(n)
        for s in range(len(boxes)):
            out[own == s] = fields[s][own == s]
        return out

    for _ in range(steps):
        for s in order:
            inside, art = masks[s]
            for o in range(len(boxes)):
                sel = art & (own == o)
                fields[s][sel] = fields[o][sel]
            G = glued()
            G[inside] = fields[s][inside]
            E = O.solve_single(g, mon, dt, 0.0, 1, psi0=G, theta_val=th).psi
            live = inside & ~art
            fields[s][live] = E[live]
    for s in range(len(boxes)):  # refresh before the glue
        inside, art = masks[s]
        for o in range(len(boxes)):
            sel = art & (own == o)
            fields[s][sel] = fields[o][sel]
    return glued(), fields, boxes


@pytest.mark.parametrize("n,parts,ov,mode", [
    ((25, 25), (2, 1), (4, 4), "alternating"),
    ((25, 25), (3, 1), (4, 4), "coloured"),
    ((25, 25), (2, 2), (3, 4), "alternating"),
    ((25, 29), (3, 2), (4, 3), "alternating"),
    ((25, 29), (3, 2), (4, 3), "coloured"),
    ((13, 13, 13), (2, 1, 2), (3, 3, 3), "alternating"),
])
def test_alternating_euler_equals_whole_domain_steps(n, parts, ov, mode):
    g = O.GridSpec(n, (0.0,) * len(n), (1.0,) * len(n))
    mon = W.ring_monitor(d=len(n))
    dt, steps = 2e-4, 4
    r = O.solve_dd(g, parts, ov, mon, dt, 0.0, steps, mode=mode)
    dec = O.Decomposition(g, parts, ov)
    order = O.sweep_order(dec, mode)
    want, fields, boxes = _alternating_by_whole_domain_steps(g, parts, ov, mon, dt, steps, order)
    np.testing.assert_array_equal(r.psi, want)
    for s, b in enumerate(boxes):
        sl = tuple(slice(lo, hi + 1) for lo, hi in b)
        np.testing.assert_array_equal(r.sub_psi[s], fields[s][sl])
    # reading the owners' newest values matters: the parallel form differs
    par = O.solve_dd(g, parts, ov, mon, dt, 0.0, steps)
    assert np.max(np.abs(par.psi - r.psi)) > 1e-12


def test_sweep_orders():
    dec = O.Decomposition(O.GridSpec((33, 33), (0.0, 0.0), (1.0, 1.0)), (4, 1), (4, 4))
    assert O.sweep_order(dec, "alternating") == [0, 1, 2, 3]
    assert O.sweep_order(dec, "coloured") == [0, 2, 1, 3]
    dec = O.Decomposition(O.GridSpec((33, 33), (0.0, 0.0), (1.0, 1.0)), (3, 3), (4, 4))
    assert O.sweep_order(dec, "coloured") == [0, 2, 6, 8, 1, 7, 3, 5, 4]
    # 2 x 2 (x 2): every parity class is one subdomain, so both orders are the block order
    for shape, parts in (((17, 17), (2, 2)), ((9, 9, 9), (2, 2, 2))):
        dec = O.Decomposition(O.GridSpec(shape, (0.0,) * len(shape), (1.0,) * len(shape)), parts, (3,) * len(shape))
        assert O.sweep_order(dec, "coloured") == O.sweep_order(dec, "alternating")


def _alternating_1d_bruteforce(n, parts, ov, A, K, C, dt, gamma, steps, order):
    """1D alternating DD by loops: Neumann ghosts Psi_{-1} = Psi_1 - 2 h a, Psi_{N+1} =
    Psi_{N-1} + 2 h b at the physical ends, F = log(rho(Psi') Psi'' / theta) with the exact
    theta of 1 + A sech^2(K (x - C)) on [0, 1], and (I - gamma L) delta = F solved with the
    assembled subdomain matrix (Neumann reflection at both ends of the subdomain)."""
    h = 1.0 / (n - 1)
    xi = np.linspace(0.0, 1.0, n)
    cores, ranges = O.partition_axis(n - 1, parts, ov)
    own = O.owner_axis(np.arange(n), cores)
    th = 1.0 + (A / K) * (math.tanh(K * (1.0 - C)) - math.tanh(K * (0.0 - C)))
    states = [0.5 * xi[lo:hi + 1] ** 2 for lo, hi in ranges]

    def refresh(m):
        lo, hi = ranges[m]
        for v in (lo, hi):
            if 0 < v < n - 1:
                o = own[v]
                states[m][v - lo] = states[o][v - ranges[o][0]]

    for _ in range(steps):
        for m in order:
            refresh(m)
            lo, hi = ranges[m]
            P = states[m]
            L = len(P)
            F = np.zeros(L)
            for j in range(L):
                v = lo + j
                if (j == 0 and v > 0) or (j == L - 1 and v < n - 1):
                    continue
                left = P[j - 1] if j > 0 else P[1] - 2.0 * h * 0.0
                right = P[j + 1] if j < L - 1 else P[j - 1] + 2.0 * h * 1.0
                d1 = (right - left) / (2.0 * h)
                d2 = (right - 2.0 * P[j] + left) / (h * h)
                rho = 1.0 + A / math.cosh(K * (d1 - C)) ** 2
                F[j] = math.log(rho * d2 / th)
            M = np.eye(L)
            for j in range(L):
                M[j, j] += 2.0 * gamma / (h * h)
                if j > 0:
                    M[j, j - 1] -= (2.0 if j == L - 1 else 1.0) * gamma / (h * h)
                if j < L - 1:
                    M[j, j + 1] -= (2.0 if j == 0 else 1.0) * gamma / (h * h)
            delta = np.linalg.solve(M, F)
            for j in range(L):
                v = lo + j
                if not ((j == 0 and v > 0) or (j == L - 1 and v < n - 1)):
                    P[j] += dt * delta[j]
    for m in range(len(ranges)):
        refresh(m)
    out = np.empty(n)
    for v in range(n):
        o = own[v]
        out[v] = states[o][v - ranges[o][0]]
    return out


@pytest.mark.parametrize("parts,mode", [(2, "alternating"), (3, "alternating"), (4, "coloured")])
def test_alternating_1d_matches_bruteforce(parts, mode):
    n, ov, A, K, C = 41, 4, 6.0, 12.0, 0.37
    h = 1.0 / (n - 1)
    gamma, dt, steps = 4 * h * h, 0.8 * h * h, 12
    g1 = O.GridSpec((n,), (0.0,), (1.0,))
    r = O.solve_dd(g1, (parts,), (ov,), W.separable_monitor((A,), (K,), (C,)), dt, gamma, steps, mode=mode)
    order = O.sweep_order(O.Decomposition(g1, (parts,), (ov,)), mode)
    want = _alternating_1d_bruteforce(n, parts, ov, A, K, C, dt, gamma, steps, order)
    assert np.max(np.abs(r.psi - want)) < 1e-13


# --- Arc-length monitors of the paper's test functions (Sec. 4, eq. monitfn) -----------------

def _u_front(X, eps, s0):
    return 1.0 / (1.0 + np.exp((X[..., 0] + X[..., 1] - s0) / (2.0 * eps)))


def _u_spiral(X, A, k, w, c):
    dx, dy = X[..., 0] - c[0], X[..., 1] - c[1]
    r2 = dx * dx + dy * dy
    return 1.0 + A / (1.0 + k * r2 * np.cos(np.arctan2(dy, dx) - w * r2) ** 2)


def _u_spheres(X, k, r0, centres):
    out = np.zeros(X.shape[:-1])
    for c in centres:
        out = out + np.tanh(k * (np.sum((X - np.asarray(c)) ** 2, axis=-1) - r0 * r0))
    return out


def _fd_gradient(u, X, h):
    """Fourth-order central differences of u at the points X[..., d]."""
    G = np.zeros(X.shape)
    for q in range(X.shape[-1]):
        e = np.zeros(X.shape[-1])
        e[q] = h
        G[..., q] = (-u(X + 2 * e) + 8 * u(X + e) - 8 * u(X - e) + u(X - 2 * e)) / (12 * h)
    return G


@pytest.mark.parametrize("case", ["front", "spiral", "sphere", "spheres9"])
def test_arclen_gradient_matches_finite_differences(case):
    # the monitor's grad u is derived by hand; u itself is the paper's formula
    rng = np.random.default_rng(7)
    if case == "front":
        mon = W.front_monitor(eps=0.05)
        X = rng.uniform(0.0, 1.0, (400, 2))
        u = lambda Y: _u_front(Y, 0.05, 1.0)
    elif case == "spiral":
        mon = W.spiral_monitor()
        X = rng.uniform(0.0, 1.0, (400, 2))
        u = lambda Y: _u_spiral(Y, 9.0, 100.0, 20.0, (0.7, 0.5))
    elif case == "sphere":
        mon = W.spheres_monitor(100.0, math.sqrt(0.125), [(0.0, 0.0, 0.0)])
        X = rng.uniform(-0.6, 0.6, (400, 3))
        u = lambda Y: _u_spheres(Y, 100.0, math.sqrt(0.125), [(0.0, 0.0, 0.0)])
    else:
        mon = W.spheres_monitor(50.0, math.sqrt(0.1875), W.NINE_CENTRES)
        X = rng.uniform(-1.2, 1.2, (400, 3))
        u = lambda Y: _u_spheres(Y, 50.0, math.sqrt(0.1875), W.NINE_CENTRES)
    G = O.grad_u(mon, X)
    F = _fd_gradient(u, X, 3e-5)
    scale = np.max(np.abs(F), axis=-1, keepdims=True) + 1.0
    assert np.max(np.abs(G - F) / scale) < 1e-6
    np.testing.assert_allclose(O.rho(mon, X), np.sqrt(1.0 + np.sum(F * F, axis=-1)), rtol=1e-6)


def test_arclen_front_theta_reduction_equals_tensor_quadrature():
    mon = W.front_monitor(eps=0.01)
    for lo, hi in (((0.0, 0.0), (1.0, 1.0)), ((-0.2, 0.1), (1.3, 0.9))):
        red = O.theta_reduced(mon, lo, hi)
        quad = O.theta_quadrature(mon, lo, hi)
        assert abs(red - quad) < 1e-11 * quad, (red, quad)


@pytest.mark.parametrize("d", [2, 3])
def test_arclen_sphere_theta_radial_reduction_equals_tensor_quadrature(d):
    # a broad shell so that the tensor rule converges quickly; the reduction needs the shell's
    # tail inside the box
    mon = W.spheres_monitor(10.0, 0.4, [(0.1, -0.2, 0.05)[:d]])
    lo, hi = (-3.0,) * d, (3.2,) * d
    red = O.theta_reduced(mon, lo, hi)
    assert red is not None
    quad = O.theta_quadrature(mon, lo, hi, panels=48 if d == 3 else 200)
    assert abs(red - quad) < 1e-9 * quad, (red, quad)
    assert O.theta_reduced(mon, (-1.0,) * d, (1.0,) * d) is None  # tail leaves the box


def test_arclen_spiral_theta_converged():
    # the ridges of the spiral reach rho ~ 1.7e3 over widths ~ 3e-3 near the far corner; the
    # tensor rule settles to ~1e-7 relative (theta only adds a constant to F)
    mon = W.spiral_monitor()
    a = O.theta_quadrature(mon, (0.0, 0.0), (1.0, 1.0))
    b = O.theta_quadrature(mon, (0.0, 0.0), (1.0, 1.0), panels=int(1.5 * O.pma_oracle._panels_for(mon, (0.0, 0.0), (1.0, 1.0))))
    assert abs(a - b) < 3e-7 * a, (a, b)


def test_arclen_front_mesh_symmetries():
    # u depends on x + y and is odd about the line x + y = 1, so rho is invariant under the swap
    # of axes and under (x, y) -> (1 - y, 1 - x): the mesh inherits both
    g = grid2(33)
    r = O.solve_single(g, W.front_monitor(eps=0.03), 1e-3, 1.0, 60)
    x, y = r.mesh
    assert np.max(np.abs(x - y.T)) < 1e-12
    assert np.max(np.abs(x - (1.0 - y[::-1, ::-1].T))) < 1e-12
    assert r.min_det > 0 and r.min_cell > 0


def test_arclen_nine_spheres_mesh_cube_symmetry():
    # the nine centres are invariant under every permutation and sign flip of the axes
    g = O.GridSpec((13, 13, 13), (-2.0,) * 3, (2.0,) * 3)
    mon = dict(W.spheres_monitor(5.0, math.sqrt(0.1875), W.NINE_CENTRES), theta=70.0)
    r = O.solve_single(g, mon, 1e-3, 1.0, 20)
    x = r.mesh
    assert np.max(np.abs(x[0] - np.transpose(x[1], (1, 0, 2)))) < 1e-12
    assert np.max(np.abs(x[0] - np.transpose(x[2], (2, 1, 0)))) < 1e-12
    assert np.max(np.abs(x[0] + x[0][::-1, :, :])) < 1e-12
    assert r.min_det > 0


# --- Jacobian check (a8): min det D^2_h Psi, pinned by closed forms ---------------------------

def _box_of(n, lo, hi, art=False):
    d = len(n)
    h = tuple((b - a) / (k - 1) for a, b, k in zip(lo, hi, n))
    return O.Box((0,) * d, tuple(n), h, tuple(lo), tuple(hi), (art,) * d, (art,) * d)


@pytest.mark.parametrize("n,lo,hi", [((17, 11), (0.0, -1.0), (2.0, 0.5)), ((9, 7, 8), (-1.0, 0.0, 0.5), (1.0, 3.0, 1.0))])
def test_min_det_hessian_of_initial_potential_is_one(n, lo, hi):
    # Psi^0 = |xi|^2 / 2 (eq. incond): centred differences are exact for quadratics, and the
    # Neumann ghost of eq. nbd reproduces the quadratic, so D^2_h Psi = I at every node
    box = _box_of(n, lo, hi)
    assert abs(O.min_det_hessian(O.initial_psi(box), box) - 1.0) < 1e-12


@pytest.mark.parametrize("n,lo,hi,eps,m", [
    ((33, 21), (0.0, -1.0), (2.0, 0.5), (0.02, 0.008), (2, 1)),
    ((17, 13, 15), (-1.0, 0.0, 0.5), (1.0, 2.0, 1.5), (0.01, 0.02, 0.004), (1, 1, 1))])
def test_min_det_hessian_cosine_perturbation_closed_form(n, lo, hi, eps, m):
    # Psi = sum_k xi_k^2 / 2 + eps_k cos(w_k (xi_k - a_k)), w_k = 2 pi m_k / (b_k - a_k).  The
    # cosine is even about both faces, so the centred Neumann ghost is exact; the discrete second
    # difference of cos(w s) is -lam cos(w s) with lam = (4 / h^2) sin^2(w h / 2), and the cross
    # differences of a separable function vanish.  So D^2_h Psi = diag(1 - eps_k lam_k cos(..)),
    # whose smallest determinant sits where every cosine is 1 (the low corner):
    # prod_k (1 - eps_k lam_k).
    box = _box_of(n, lo, hi)
    d = len(n)
    X = box.coords()
    psi = 0.5 * np.sum(X * X, axis=-1)
    expect = 1.0
    for k in range(d):
        w = 2.0 * math.pi * m[k] / (hi[k] - lo[k])
        psi = psi + eps[k] * np.cos(w * (X[..., k] - lo[k]))
        lam = 4.0 / box.h[k] ** 2 * math.sin(w * box.h[k] / 2.0) ** 2
        assert eps[k] * lam < 0.9
        expect *= 1.0 - eps[k] * lam
    got = O.min_det_hessian(psi, box)
    assert abs(got - expect) < 1e-9, (got, expect)


def test_det_sym_3d_matches_numpy_det():
    rng = np.random.default_rng(7)
    M = rng.standard_normal((50, 3, 3))
    M = M + np.transpose(M, (0, 2, 1))
    hess = [[M[:, i, j] for j in range(3)] for i in range(3)]
    np.testing.assert_allclose(O.det_sym(hess, 3), np.linalg.det(M), rtol=1e-12, atol=1e-12)
    hess2 = [[M[:, i, j] for j in range(2)] for i in range(2)]
    np.testing.assert_allclose(O.det_sym(hess2, 2), np.linalg.det(M[:, :2, :2]), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("d", [2, 3])
def test_min_det_hessian_quadratic_with_mixed_terms(d):
    # Psi = xi^T M xi / 2 + b . xi on a box whose faces are all artificial (live nodes are the
    # interior ones, whose stencils use real values only): every second and mixed difference is
    # exact for a quadratic, so det D^2_h Psi = det M (numpy.linalg.det) at every live node
    rng = np.random.default_rng(11 + d)
    A = rng.standard_normal((d, d))
    M = A @ A.T + d * np.eye(d)
    b = rng.standard_normal(d)
    n = (9, 8, 7)[:d]
    box = _box_of(n, (-0.5,) * d, (1.5,) * d, art=True)
    X = box.coords()
    psi = 0.5 * np.einsum("...i,ij,...j->...", X, M, X) + X @ b
    assert abs(O.min_det_hessian(psi, box) - np.linalg.det(M)) < 1e-9 * np.linalg.det(M)


# --- relative errors of Sec. 4.4 (eqs. rel_errlp / rel_errlinf) with the trapezoid rule ---------

@pytest.mark.parametrize("n", [(9, 5), (17, 3)])
def test_rel_errors_closed_forms(n):
    # on [0, 2] x [0, 1]: Psi_sd = 1, Psi_dd = 1 - xi.  The trapezoid rule integrates 1 and xi
    # exactly (2 and 2), and xi^2 to 8/3 + h^2/3 (its error term for a constant second derivative)
    lo, hi = (0.0, 0.0), (2.0, 1.0)
    g = O.GridSpec(n, lo, hi)
    X = g.whole_box().coords()
    ref = np.ones(n)
    approx = ref - X[..., 0]
    e = O.rel_errors(ref, approx, g.h)
    h0 = g.h[0]
    assert abs(e[1] - 2.0 / 2.0) < 1e-13
    assert abs(e[2] - math.sqrt((8.0 / 3.0 + h0 * h0 / 3.0) / 2.0)) < 1e-13
    assert abs(e["inf"] - 2.0) < 1e-13
    # the relative form divides by the norm of the reference: scaling both leaves E unchanged
    e3 = O.rel_errors(3.0 * ref, 3.0 * approx, g.h)
    for p in (1, 2, "inf"):
        assert abs(e3[p] - e[p]) < 1e-13


# --- residual of eq. dd_stop_criterion: closed forms -----------------------------------------

@pytest.mark.parametrize("n,lo,hi", [((9, 13), (0.0, -1.0), (2.0, 2.0)), ((5, 7, 6), (0.0, 0.0, -1.0), (1.0, 3.0, 1.0))])
def test_residual_closed_form_constant_update(n, lo, hi):
    # constant monitor, Psi^0 = |xi|^2 / 2 (det D^2_h Psi = 1) and theta = |Omega| amp e^{-c}:
    # F = c at every node, and with gamma = 0 the update is dt c everywhere, whose trapezoid L2
    # norm is dt |c| |Omega|^{1/2}
    g = O.GridSpec(n, lo, hi)
    box = g.whole_box()
    amp, c, dt = 3.0, 0.37, 1e-3
    mon = W.const_monitor(amp)
    th = g.vol * amp * math.exp(-c)
    psi1, res = O.step_box(O.initial_psi(box), box, mon, th, g.vol, dt, 0.0)
    assert abs(res - dt * c * math.sqrt(g.vol)) < 1e-15
    assert np.max(np.abs(psi1 - O.initial_psi(box) - dt * c)) < 1e-15
    # the preconditioner keeps a constant (its DC mode has mu_0 = 0)
    psi1p, resp = O.step_box(O.initial_psi(box), box, mon, th, g.vol, dt, 0.5)
    assert abs(resp - dt * c * math.sqrt(g.vol)) < 1e-14


@pytest.mark.parametrize("n", [(9, 13), (5, 7, 6)])
def test_residual_excludes_artificial_nodes(n):
    # a box with every face artificial: only interior nodes are live, each of trapezoid weight
    # prod h, so the norm of a constant update dt c is dt |c| (prod_k (n_k - 2) h_k)^{1/2}
    d = len(n)
    box = _box_of(n, (0.0,) * d, (2.0,) * d, art=True)
    vol = 2.0 ** d
    amp, c, dt = 2.0, -0.21, 1e-3
    th = vol * amp * math.exp(-c)
    _, res = O.step_box(O.initial_psi(box), box, W.const_monitor(amp), th, vol, dt, 0.0)
    expect = dt * abs(c) * math.sqrt(float(np.prod([(k - 2) * hk for k, hk in zip(n, box.h)])))
    assert abs(res - expect) < 1e-15


# --- quality measure of Sec. 4.5: a mesh with a closed-form Jacobian --------------------------

@pytest.mark.parametrize("n,lo,hi,eps", [((11, 9), (0.0, -1.0), (2.0, 0.0), (0.2, 0.5)),
                                         ((7, 9, 5), (0.0, 0.0, -1.0), (1.0, 2.0, 1.0), (0.3, 0.1, 0.2))])
def test_quality_of_mesh_closed_form(n, lo, hi, eps):
    # x_k = xi_k + eps_k (xi_k - a_k)(b_k - xi_k): dx_k/dxi_k = 1 + eps_k (a_k + b_k - 2 xi_k) is
    # linear, so second-order differences (one-sided at the faces) give it exactly and
    # J = prod_k (1 + eps_k (a_k + b_k - 2 xi_k)).  With a constant monitor E = J, whose maximum
    # is prod_k (1 + eps_k L_k) at the low corner, and whose trapezoid integral of E^2 is
    # prod_k [L_k (1 + eps_k^2 L_k^2 / 3) + (2/3) eps_k^2 L_k h_k^2] (exact part plus the rule's
    # error term for a quadratic)
    g = O.GridSpec(n, lo, hi)
    d = len(n)
    X = g.whole_box().coords()
    mesh = np.stack([X[..., k] + eps[k] * (X[..., k] - lo[k]) * (hi[k] - X[..., k]) for k in range(d)], 0)
    mon = W.const_monitor(1.7)
    q = O.quality_of_mesh(mesh, g, mon, theta_val=1.7 * g.vol)
    L = [b - a for a, b in zip(lo, hi)]
    emax = float(np.prod([1.0 + e * l for e, l in zip(eps, L)]))
    int2 = float(np.prod([l * (1.0 + e * e * l * l / 3.0) + 2.0 / 3.0 * e * e * l * h * h
                          for e, l, h in zip(eps, L, g.h)]))
    assert abs(q["Emax"] - emax) < 1e-12
    assert abs(q["E2"] - math.sqrt(int2 / g.vol)) < 1e-12


def test_negative_monitor_raises_nonfinite():
    # rho = 1 - 5 exp(-|x - c|^2 / (2 w^2)) < 0 near c with theta given positive: no real log
    g = grid2(17)
    mon = {"kind": "gauss_sum", "bamp": [-5.0], "bw": [0.1], "bc": [[0.5, 0.5]]}
    with pytest.raises(O.NonFiniteError):
        O.solve_single(g, mon, 1e-3, 1.0, 3, theta_val=1.0)
    # the same bump with a positive amplitude runs
    O.solve_single(g, dict(mon, bamp=[5.0]), 1e-3, 1.0, 3)
