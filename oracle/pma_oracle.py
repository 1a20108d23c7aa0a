"""Plain FP64 CPU oracle for the (domain-decomposition) parabolic Monge-Ampere mesh method.

TEST INFRASTRUCTURE ONLY.  This module is the correctness authority that the GPU path is
checked against.  Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product library never does, and the two share no code.

Everything here is slow, vectorised NumPy in float64, written to be read against the paper
(Sulman, Nguyen, Haynes, Huang, "Domain decomposition parabolic Monge-Ampere approach for fast
generation of adaptive moving meshes", arXiv 2006.14602).  Section / equation references below
are to that paper.

State is the potential Psi itself (the paper's form), dimension d in {1, 2, 3}.  Arrays are
indexed [i0, i1, i2] with axis k the k-th coordinate; node i on axis k sits at
xi_k = a_k + i * h_k, h_k = (b_k - a_k) / N_k.

Readings of points the paper leaves open (listed again in the design notes):
  * Neumann condition grad Psi . n = xi . n (Sec. 2, eq. nbd) by one ghost layer from the
    centred difference: Psi_{-1} = Psi_1 - 2 h a, Psi_{N+1} = Psi_{N-1} + 2 h b; axes are
    padded in turn so corner ghosts get both reflections.
  * "standard centered finite differences" (Sec. 3, eqs. pmae1d/pmae2d): centred first
    differences, 3-point second differences, 4-point cross for mixed second differences.
  * rho is normalised by theta = int_Omega rho (Sec. 2, text before eq. edp), so the right
    hand side is log(|Omega_c| rho det D^2 Psi / theta).
  * Time integration: the paper integrates each step with a variable-order ODE solver and uses
    forward Euler for its time-convergence study (Sec. 4.4).  Here one step is
        (I - gamma L_h) delta = F(Psi^n),   Psi^{n+1} = Psi^n + dt * delta,
    L_h the Neumann Laplacian with ghost reflection; gamma = 0 is forward Euler exactly.
  * Parallel DD (Sec. 3, eq. transmission_condition3): at the start of each step every
    artificial-boundary node takes its owner's time-n value and holds it through the step.
  * Subdomain preconditioner: homogeneous Neumann on every subdomain face; F := 0 and no update
    on artificial-boundary nodes.
  * Stop rule (Algorithm 1, step 6): the maximum over subdomains (all converged) by default.
  * Alternating DD (Algorithm 1) with more than two subdomains: the subdomains are updated one
    after another within a step, each first taking its artificial-boundary values from the
    owners' latest values (time n+1 for owners already updated in this step, time n for the
    rest).  The sweep order is the lexicographic order of the block index ("alternating"), or
    the 2^d parity classes of the block index in lexicographic order of the parity tuple, each
    class in block order ("coloured").  With two subdomains both are Algorithm 1 exactly.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.fft
import scipy.optimize
import scipy.special


class TangledError(ArithmeticError):
    """det D^2_h Psi <= 0 somewhere: log of a non-positive number (the mesh has folded)."""


class NonFiniteError(ArithmeticError):
    """The right-hand side of eq. pmae is not a finite real number somewhere (a monitor that is
    not positive, or an overflow): the log has no real value."""


# ----------------------------------------------------------------------------------------
# Monitor functions rho(x).  A monitor is a plain dict (see the workload generators).
# ----------------------------------------------------------------------------------------

def _sech2(z):
    """sech^2(z) = 4 e^{-2|z|} / (1 + e^{-2|z|})^2, overflow-free."""
    e = np.exp(-2.0 * np.abs(z))
    return 4.0 * e / (1.0 + e) ** 2


def rho(mon: dict, X: np.ndarray) -> np.ndarray:
    """Evaluate the monitor at physical points X[..., d] (float64)."""
    kind = mon["kind"]
    d = X.shape[-1]
    if kind == "const":
        return np.full(X.shape[:-1], float(mon.get("amp", 1.0)))
    if kind == "sech2_radial":
        # 1 + A sech^2(k (|x - c|^2 - r0^2))
        c = np.asarray(mon["c"], dtype=np.float64)[:d]
        r2 = np.sum((X - c) ** 2, axis=-1)
        return 1.0 + mon["amp"] * _sech2(mon["k"] * (r2 - mon["r0"] ** 2))
    if kind == "sech2_sine":
        # 1 + A sech^2(k (x_1 - c_1 - r0 sin(2 pi x_0)))   (a sine-wave layer)
        c1 = float(np.asarray(mon["c"], dtype=np.float64)[1])
        s = X[..., 1] - c1 - mon["r0"] * np.sin(2.0 * np.pi * X[..., 0])
        return 1.0 + mon["amp"] * _sech2(mon["k"] * s)
    if kind == "gauss_sum":
        # 1 + sum_b A_b exp(-|x - c_b|^2 / (2 w_b^2))
        out = np.ones(X.shape[:-1])
        for amp, w, c in zip(mon["bamp"], mon["bw"], mon["bc"]):
            c = np.asarray(c, dtype=np.float64)[:d]
            out = out + amp * np.exp(-np.sum((X - c) ** 2, axis=-1) / (2.0 * w * w))
        return out
    if kind == "separable_sech2":
        # prod_k (1 + A_k sech^2(k_k (x_k - c_k)))
        out = np.ones(X.shape[:-1])
        for ax in range(d):
            out = out * (1.0 + mon["amp_axes"][ax] * _sech2(mon["k_axes"][ax] * (X[..., ax] - mon["c"][ax])))
        return out
    if kind in ARCLEN_KINDS:
        # arc-length monitor of a given solution u (Sec. 4, eq. monitfn)
        G = grad_u(mon, X)
        return np.sqrt(1.0 + np.sum(G * G, axis=-1))
    raise ValueError(f"unknown monitor kind {kind!r}")


ARCLEN_KINDS = ("arclen_front", "arclen_spiral", "arclen_spheres")


def grad_u(mon: dict, X: np.ndarray) -> np.ndarray:
    """Gradient of the physical solution u behind an arc-length monitor, at X[..., d].

    arclen_front   u = 1 / (1 + exp((x_0 + x_1 - s0) / (2 eps)))      (Sec. 4.1, eq. test_fn1)
    arclen_spiral  u = 1 + A / (1 + k r^2 cos^2(theta - w r^2)), r and theta polar coordinates
                   about c                                             (Sec. 4.1, eq. test_fn2)
    arclen_spheres u = sum_b tanh(k (|x - c_b|^2 - r0^2))   (Sec. 4.2, eqs. test_fn3d1/test_fn3d2)
    """
    kind = mon["kind"]
    d = X.shape[-1]
    G = np.zeros(X.shape)
    if kind == "arclen_front":
        eps, s0 = float(mon["eps"]), float(mon.get("offset", 1.0))
        s = (X[..., 0] + X[..., 1] - s0) / (2.0 * eps)
        u = scipy.special.expit(-s)
        du = -u * (1.0 - u) / (2.0 * eps)       # du/dx_0 = du/dx_1
        G[..., 0] = du
        G[..., 1] = du
        return G
    if kind == "arclen_spiral":
        A, k, w = float(mon["amp"]), float(mon["k"]), float(mon["twist"])
        dx, dy = X[..., 0] - mon["c"][0], X[..., 1] - mon["c"][1]
        r = np.hypot(dx, dy)
        th = np.arctan2(dy, dx)
        phi = th - w * r * r
        q = k * r * r * np.cos(phi) ** 2
        # q = k r^2 cos^2(phi), phi = theta - w r^2:
        #   dq/dr = 2 k r (cos^2 phi + w r^2 sin 2 phi),  (1/r) dq/dtheta = -k r sin 2 phi
        dq_dr = 2.0 * k * r * (np.cos(phi) ** 2 + w * r * r * np.sin(2.0 * phi))
        dq_t = -k * r * np.sin(2.0 * phi)
        f = -A / (1.0 + q) ** 2
        G[..., 0] = f * (dq_dr * np.cos(th) - dq_t * np.sin(th))
        G[..., 1] = f * (dq_dr * np.sin(th) + dq_t * np.cos(th))
        return G
    if kind == "arclen_spheres":
        k, r02 = float(mon["k"]), float(mon["r0"]) ** 2
        for c in mon["bc"]:
            D = X - np.asarray(c, dtype=np.float64)[:d]
            g = 2.0 * k * _sech2(k * (np.sum(D * D, axis=-1) - r02))
            G = G + g[..., None] * D
        return G
    raise ValueError(f"no solution u for monitor kind {kind!r}")


# ----------------------------------------------------------------------------------------
# theta = int_Omega rho dx  (normalisation, Sec. 2 text before eq. edp)
# ----------------------------------------------------------------------------------------

def _gauss_legendre_panels(a: float, b: float, panels: int, order: int = 8):
    t, w = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(a, b, panels + 1)
    mid = 0.5 * (edges[1:] + edges[:-1])
    half = 0.5 * (edges[1:] - edges[:-1])
    x = (mid[:, None] + half[:, None] * t[None, :]).ravel()
    wt = (half[:, None] * w[None, :]).ravel()
    return x, wt


def _panels_for(mon: dict, lo, hi) -> int:
    """Panel count per axis so that each Gauss-Legendre panel is short against the monitor's
    length scale (the distance of the nearest complex singularity of sech^2, or the Gaussian
    width)."""
    L = max(float(b - a) for a, b in zip(lo, hi))
    kind = mon["kind"]
    if kind == "sech2_radial":
        # sech^2 poles sit at k (r^2 - r0^2) = i pi / 2; near the shell dr ~ pi / (4 k r).
        scale = math.pi / (4.0 * mon["k"] * max(mon["r0"], 0.05) + 1e-300)
    elif kind == "sech2_sine":
        scale = math.pi / (2.0 * mon["k"] * (1.0 + 2.0 * math.pi * mon["r0"]))
    elif kind == "gauss_sum":
        scale = min(mon["bw"])
    elif kind == "separable_sech2":
        scale = math.pi / (2.0 * max(mon["k_axes"]))
    elif kind == "arclen_front":
        scale = math.pi * mon["eps"]
    elif kind == "arclen_spiral":
        # the ridges of u narrow to ~ 1 / (sqrt(k) 2 w r^2) away from the centre
        rmax = max(math.hypot(x - mon["c"][0], y - mon["c"][1]) for x in (lo[0], hi[0]) for y in (lo[1], hi[1]))
        scale = 1.0 / (math.sqrt(mon["k"]) * 2.0 * mon["twist"] * rmax * rmax)
    elif kind == "arclen_spheres":
        scale = math.pi / (4.0 * mon["k"] * max(mon["r0"], 0.05))
    else:
        scale = L
    return int(min(4096, max(8, math.ceil(2.0 * L / scale))))


def theta_quadrature(mon: dict, lo, hi, panels: int | None = None) -> float:
    """int_box rho dx by tensor-product composite 8-point Gauss-Legendre (float64)."""
    d = len(lo)
    if panels is None:
        panels = _panels_for(mon, lo, hi)
    nodes = [_gauss_legendre_panels(lo[k], hi[k], panels) for k in range(d)]
    total = 0.0
    # integrate over axis 0 one node at a time to bound memory
    x0, w0 = nodes[0]
    if d == 1:
        return float(np.sum(rho(mon, x0[:, None]) * w0))
    rest = np.meshgrid(*[n[0] for n in nodes[1:]], indexing="ij")
    wrest = np.ones(rest[0].shape)
    for k, n in enumerate(nodes[1:]):
        shape = [1] * (d - 1)
        shape[k] = -1
        wrest = wrest * n[1].reshape(shape)
    chunk = max(1, 2_000_000 // wrest.size)
    for s in range(0, x0.size, chunk):
        xs = x0[s:s + chunk]
        X = np.empty((xs.size,) + rest[0].shape + (d,))
        X[..., 0] = xs.reshape((-1,) + (1,) * (d - 1))
        for k in range(1, d):
            X[..., k] = rest[k - 1][None]
        vals = rho(mon, X)
        total += float(np.sum(vals * wrest[None] * w0[s:s + chunk].reshape((-1,) + (1,) * (d - 1))))
    return total


def theta_closed_form(mon: dict, lo, hi) -> float | None:
    """Exact int_box rho where it is elementary (const, Gaussian sums via erf, separable sech^2
    via tanh).  None where no closed form is known."""
    d = len(lo)
    vol = float(np.prod([b - a for a, b in zip(lo, hi)]))
    kind = mon["kind"]
    if kind == "const":
        return float(mon.get("amp", 1.0)) * vol
    if kind == "gauss_sum":
        tot = vol
        for amp, w, c in zip(mon["bamp"], mon["bw"], mon["bc"]):
            p = amp
            for k in range(d):
                s = math.sqrt(2.0) * w
                p *= w * math.sqrt(math.pi / 2.0) * (math.erf((hi[k] - c[k]) / s) - math.erf((lo[k] - c[k]) / s))
            tot += p
        return tot
    if kind == "separable_sech2":
        p = 1.0
        for k in range(d):
            A, kk, c = mon["amp_axes"][k], mon["k_axes"][k], mon["c"][k]
            p *= (hi[k] - lo[k]) + (A / kk) * (math.tanh(kk * (hi[k] - c)) - math.tanh(kk * (lo[k] - c)))
        return p
    return None


def theta_reduced(mon: dict, lo, hi) -> float | None:
    """int_box rho reduced to one dimension where the monitor allows it (adaptive quadrature):
      * arclen_front depends on s = x_0 + x_1 only: int rho = int rho(s) m(s) ds, m(s) the
        length of the segment {x_0 + x_1 = s} inside the box (the trapezoid density of the sum);
      * arclen_spheres with one centre whose shell, out to where rho - 1 < 1e-30, lies inside the
        box: vol + int_0^R (rho(r) - 1) |S^{d-1}| r^{d-1} dr.
    None where neither applies."""
    import scipy.integrate
    d = len(lo)
    vol = float(np.prod([b - a for a, b in zip(lo, hi)]))
    kind = mon["kind"]
    if kind == "arclen_front" and d == 2:
        s0 = float(mon.get("offset", 1.0))

        def m(s):
            return max(0.0, min(hi[0], s - lo[1]) - max(lo[0], s - hi[1]))

        def f(s):
            X = np.array([[s - 0.5 * s0, 0.5 * s0]])  # any point with x_0 + x_1 = s
            return float(rho(mon, X)[0]) * m(s)

        a, b = lo[0] + lo[1], hi[0] + hi[1]
        pts = sorted({a, b, lo[0] + hi[1], hi[0] + lo[1], min(max(s0, a), b)})
        tot = 0.0
        for u, v in zip(pts[:-1], pts[1:]):
            if v > u:
                tot += scipy.integrate.quad(f, u, v, epsabs=1e-14, epsrel=1e-13, limit=400,
                                            points=[s0] if u < s0 < v else None)[0]
        return tot
    if kind == "arclen_spheres" and len(mon["bc"]) == 1:
        k, r0 = float(mon["k"]), float(mon["r0"])
        c = np.asarray(mon["bc"][0], dtype=np.float64)[:d]
        R = math.sqrt(r0 * r0 + 40.0 / k)   # k (R^2 - r0^2) = 40: sech^2 < 1e-34 beyond R
        if not all(lo[q] <= c[q] - R and c[q] + R <= hi[q] for q in range(d)):
            return None
        area = 2.0 * math.pi if d == 2 else 4.0 * math.pi

        def g(r):
            X = np.zeros((1, d))
            X[0, 0] = r
            return (float(rho(dict(mon, bc=[[0.0] * d]), X)[0]) - 1.0) * area * r ** (d - 1)

        return vol + scipy.integrate.quad(g, 0.0, R, epsabs=1e-14, epsrel=1e-13, limit=400, points=[r0])[0]
    return None


def theta(mon: dict, lo, hi) -> float:
    """The normalisation constant used by the oracle's solves."""
    if "theta" in mon and mon["theta"]:
        return float(mon["theta"])
    cf = theta_closed_form(mon, lo, hi)
    if cf is None:
        cf = theta_reduced(mon, lo, hi)
    return cf if cf is not None else theta_quadrature(mon, lo, hi)


# ----------------------------------------------------------------------------------------
# Discrete operators (Sec. 3, eqs. pmae1d / pmae2d) on one box of nodes.
# ----------------------------------------------------------------------------------------

@dataclass
class Box:
    """A box of grid nodes: global node offset `off`, node counts `n`, global spacing h,
    global lower corner a and upper corner b, and which faces are artificial (DD)."""
    off: tuple
    n: tuple
    h: tuple
    a: tuple
    b: tuple
    art_lo: tuple
    art_hi: tuple

    @property
    def d(self):
        return len(self.n)

    def axes(self):
        return [self.a[k] + (self.off[k] + np.arange(self.n[k])) * self.h[k] for k in range(self.d)]

    def coords(self):
        return np.stack(np.meshgrid(*self.axes(), indexing="ij"), axis=-1)

    def artificial_mask(self):
        m = np.zeros(self.n, dtype=bool)
        for k in range(self.d):
            idx = [slice(None)] * self.d
            if self.art_lo[k]:
                idx[k] = 0
                m[tuple(idx)] = True
            if self.art_hi[k]:
                idx[k] = self.n[k] - 1
                m[tuple(idx)] = True
        return m

    def trapezoid_weights(self):
        w = np.ones(self.n)
        for k in range(self.d):
            wk = np.ones(self.n[k])
            wk[0] = wk[-1] = 0.5
            shape = [1] * self.d
            shape[k] = -1
            w = w * wk.reshape(shape)
        return w * float(np.prod(self.h))


def ghost_pad(psi: np.ndarray, box: Box) -> np.ndarray:
    """Add one ghost layer per axis.  On a physical face the ghost follows from the centred
    Neumann condition (eq. nbd): Psi_{-1} = Psi_1 - 2 h a at xi = a and
    Psi_{N+1} = Psi_{N-1} + 2 h b at xi = b.  Axes are padded in turn, so corner ghosts get both
    reflections.  Artificial faces need no ghost (F is not evaluated there); they get a copy
    of the edge value so the array stays finite."""
    P = psi
    for k in range(box.d):
        n = P.shape[k]
        lo_face = [slice(None)] * P.ndim
        hi_face = [slice(None)] * P.ndim
        if box.art_lo[k]:
            lo_face[k] = slice(0, 1)
            g_lo = P[tuple(lo_face)]
        else:
            lo_face[k] = slice(1, 2)
            g_lo = P[tuple(lo_face)] - 2.0 * box.h[k] * box.a[k]
        if box.art_hi[k]:
            hi_face[k] = slice(n - 1, n)
            g_hi = P[tuple(hi_face)]
        else:
            hi_face[k] = slice(n - 2, n - 1)
            g_hi = P[tuple(hi_face)] + 2.0 * box.h[k] * box.b[k]
        P = np.concatenate([g_lo, P, g_hi], axis=k)
    return P


def _shift(P: np.ndarray, d: int, offs) -> np.ndarray:
    """View of the padded array P shifted by offs[k] in {-1, 0, 1} along each axis."""
    idx = tuple(slice(1 + o, P.shape[k] - 1 + o) for k, o in enumerate(offs))
    return P[idx]


def derivatives(psi: np.ndarray, box: Box):
    """Centred gradient and Hessian of Psi at every node of the box, using ghosts."""
    d = box.d
    P = ghost_pad(psi, box)
    z = [0] * d
    C = _shift(P, d, z)
    grad = []
    hess = [[None] * d for _ in range(d)]
    for k in range(d):
        e = list(z)
        e[k] = 1
        m = list(z)
        m[k] = -1
        Pp, Pm = _shift(P, d, e), _shift(P, d, m)
        grad.append((Pp - Pm) / (2.0 * box.h[k]))
        hess[k][k] = (Pp - 2.0 * C + Pm) / (box.h[k] ** 2)
    for k in range(d):
        for l in range(k + 1, d):
            def s(ok, ol):
                o = list(z)
                o[k] = ok
                o[l] = ol
                return _shift(P, d, o)
            hess[k][l] = (s(1, 1) - s(1, -1) - s(-1, 1) + s(-1, -1)) / (4.0 * box.h[k] * box.h[l])
            hess[l][k] = hess[k][l]
    return grad, hess


def det_sym(hess, d: int) -> np.ndarray:
    if d == 1:
        return hess[0][0]
    if d == 2:
        return hess[0][0] * hess[1][1] - hess[0][1] * hess[1][0]
    a, b, c = hess[0][0], hess[0][1], hess[0][2]
    e, f, i = hess[1][1], hess[1][2], hess[2][2]
    return a * (e * i - f * f) - b * (b * i - f * c) + c * (b * f - e * c)


def rhs_F(psi: np.ndarray, box: Box, mon: dict, theta_val: float, vol: float):
    """F = log(|Omega_c| rho(grad_h Psi) det D^2_h Psi / theta)  (eq. pmae with the
    normalisation of eq. edp), F := 0 on artificial-boundary nodes.  Raises TangledError where
    the determinant is not positive, NonFiniteError where F is not a finite real number."""
    grad, hess = derivatives(psi, box)
    det = det_sym(hess, box.d)
    art = box.artificial_mask()
    live = ~art
    if np.any(~(det[live] > 0.0)):
        raise TangledError("det D^2_h Psi <= 0")
    X = np.stack(grad, axis=-1)
    F = np.zeros(psi.shape)
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        F[live] = np.log(vol * rho(mon, X[live]) * det[live] / theta_val)
    if not np.all(np.isfinite(F)):
        raise NonFiniteError("F is not finite")
    return F


def neumann_mu(n: int, h: float) -> np.ndarray:
    """Eigenvalues of -L_h (1D, ghost-reflection Neumann) on n nodes: (4/h^2) sin^2(pi k / 2N)."""
    N = n - 1
    k = np.arange(n)
    return (4.0 / h ** 2) * np.sin(np.pi * k / (2.0 * N)) ** 2


def precondition(F: np.ndarray, h, gamma: float) -> np.ndarray:
    """Solve (I - gamma L_h) delta = F with homogeneous Neumann (ghost reflection) on every
    face.  L_h is diagonalised by the type-I DCT; gamma = 0 returns F (forward Euler)."""
    if gamma == 0.0:
        return F.copy()
    Y = scipy.fft.dctn(F, type=1)
    denom = np.ones(F.shape)
    for k in range(F.ndim):
        shape = [1] * F.ndim
        shape[k] = -1
        denom = denom + gamma * neumann_mu(F.shape[k], h[k]).reshape(shape)
    return scipy.fft.idctn(Y / denom, type=1)


def assemble_neumann_laplacian_1d(n: int, h: float):
    """Sparse 1D L_h with ghost reflection (rows 0 and N have 2(u_1 - u_0)/h^2)."""
    import scipy.sparse as sp
    main = np.full(n, -2.0)
    up = np.ones(n - 1)
    lo = np.ones(n - 1)
    up[0] = 2.0
    lo[-1] = 2.0
    return sp.diags([lo, main, up], [-1, 0, 1], format="csr") / h ** 2


# ----------------------------------------------------------------------------------------
# Grids, partition and ownership (Sec. 3: overlapping slab / block splits).
# ----------------------------------------------------------------------------------------

@dataclass
class GridSpec:
    n: tuple            # nodes per axis
    lo: tuple           # box lower corner
    hi: tuple           # box upper corner

    @property
    def d(self):
        return len(self.n)

    @property
    def N(self):
        return tuple(k - 1 for k in self.n)

    @property
    def h(self):
        return tuple((b - a) / N for a, b, N in zip(self.lo, self.hi, self.N))

    @property
    def vol(self):
        return float(np.prod([b - a for a, b in zip(self.lo, self.hi)]))

    def whole_box(self) -> Box:
        z = (False,) * self.d
        return Box((0,) * self.d, tuple(self.n), self.h, tuple(self.lo), tuple(self.hi), z, z)


def partition_axis(N: int, M: int, overlap_cells: int):
    """Cores c_m = floor(m N / M); subdomain m covers nodes
    [max(0, c_m - floor(ov/2)), min(N, c_{m+1} + ceil(ov/2))]."""
    cores = [(m * N) // M for m in range(M + 1)]
    ranges = [(max(0, cores[m] - overlap_cells // 2), min(N, cores[m + 1] + (overlap_cells + 1) // 2))
              for m in range(M)]
    return cores, ranges


def owner_axis(v: np.ndarray, cores) -> np.ndarray:
    """m with c_m <= v < c_{m+1}; the last node belongs to the last part."""
    M = len(cores) - 1
    return np.minimum(np.searchsorted(np.asarray(cores), v, side="right") - 1, M - 1)


@dataclass
class Subdomain:
    index: tuple
    box: Box
    psi: np.ndarray = field(default=None, repr=False)


class Decomposition:
    """Overlapping block split of the node grid with owners and transmission lists."""

    def __init__(self, grid: GridSpec, parts, overlap_cells):
        self.grid = grid
        d = grid.d
        self.parts = tuple(parts)
        self.axis = [partition_axis(grid.N[k], parts[k], overlap_cells[k]) for k in range(d)]
        self.subs = []
        for idx in np.ndindex(*self.parts):
            off, n, alo, ahi = [], [], [], []
            for k in range(d):
                lo_k, hi_k = self.axis[k][1][idx[k]]
                off.append(lo_k)
                n.append(hi_k - lo_k + 1)
                alo.append(lo_k > 0)
                ahi.append(hi_k < grid.N[k])
            box = Box(tuple(off), tuple(n), grid.h, tuple(grid.lo), tuple(grid.hi), tuple(alo), tuple(ahi))
            self.subs.append(Subdomain(idx, box))
        self.sub_of = {s.index: i for i, s in enumerate(self.subs)}
        self._build_transmission()

    def owner_of(self, gidx):
        """Owner subdomain number of global node index arrays gidx[k]."""
        own = [owner_axis(gidx[k], self.axis[k][0]) for k in range(self.grid.d)]
        flat = np.ravel_multi_index(own, self.parts)
        return flat

    def _build_transmission(self):
        # For every subdomain s: (dst flat index in s, src subdomain, src flat index)
        self.trans = []
        for si, s in enumerate(self.subs):
            art = s.box.artificial_mask()
            loc = np.nonzero(art)
            g = [loc[k] + s.box.off[k] for k in range(self.grid.d)]
            own = self.owner_of(g)
            lists = []
            for o in np.unique(own):
                sel = own == o
                ob = self.subs[o].box
                src_loc = [g[k][sel] - ob.off[k] for k in range(self.grid.d)]
                for k in range(self.grid.d):
                    assert np.all(src_loc[k] >= 0) and np.all(src_loc[k] < ob.n[k])
                # sources must be live (non-artificial) nodes of the owner
                assert not np.any(ob.artificial_mask()[tuple(src_loc)])
                dst = np.ravel_multi_index([loc[k][sel] for k in range(self.grid.d)], s.box.n)
                src = np.ravel_multi_index(src_loc, ob.n)
                lists.append((int(o), dst, src))
            self.trans.append(lists)

    def transmit(self, states, into=None):
        """Copy owners' values into artificial nodes.  states[s] are the arrays to read;
        writes go to `into` (default: the same arrays)."""
        into = states if into is None else into
        for si, lists in enumerate(self.trans):
            dst_flat = into[si].reshape(-1)
            for o, dst, src in lists:
                dst_flat[dst] = states[o].reshape(-1)[src]

    def glue(self, fields_per_sub):
        """Assemble a global array from per-subdomain arrays, each node from its owner."""
        d = self.grid.d
        out = np.empty(self.grid.n)
        gidx = np.meshgrid(*[np.arange(n) for n in self.grid.n], indexing="ij")
        own = self.owner_of([g.ravel() for g in gidx]).reshape(self.grid.n)
        for si, s in enumerate(self.subs):
            sel = own == si
            loc = tuple(gidx[k][sel] - s.box.off[k] for k in range(d))
            out[sel] = fields_per_sub[si][loc]
        return out


# ----------------------------------------------------------------------------------------
# Time stepping (Sec. 2 eqs. pmae/incond/nbd; Sec. 3 Algorithm 1 and eq.
# transmission_condition3).
# ----------------------------------------------------------------------------------------

def initial_psi(box: Box) -> np.ndarray:
    """Psi^0 = xi . xi / 2 (eq. incond)."""
    X = box.coords()
    return 0.5 * np.sum(X * X, axis=-1)


def step_box(psi: np.ndarray, box: Box, mon, theta_val, vol, dt, gamma):
    """One pseudo-time step on one box; returns (new psi, residual).  The residual is
    (sum_v w_v (Psi^{n+1} - Psi^n)_v^2 prod h)^{1/2} over live nodes (eq. dd_stop_criterion with
    the trapezoid rule)."""
    F = rhs_F(psi, box, mon, theta_val, vol)
    delta = precondition(F, box.h, gamma)
    live = ~box.artificial_mask()
    upd = np.where(live, dt * delta, 0.0)
    res = math.sqrt(float(np.sum(box.trapezoid_weights() * upd * upd)))
    return psi + upd, res


def mesh_from_psi(psi: np.ndarray, box: Box) -> np.ndarray:
    """x = grad_h Psi at every node (eq. adpx), shape [d, *n]."""
    grad, _ = derivatives(psi, box)
    return np.stack(grad, axis=0)


def min_det_hessian(psi: np.ndarray, box: Box) -> float:
    _, hess = derivatives(psi, box)
    det = det_sym(hess, box.d)
    live = ~box.artificial_mask()
    return float(np.min(det[live]))


def min_cell_measure(mesh: np.ndarray) -> float:
    """Minimum signed cell measure of a structured mesh x[d, *n].
    2D: area of each quadrilateral by the shoelace formula.  3D: minimum over the 8 corners of
    each hexahedron of the corner Jacobian (triple product of the three edges leaving the
    corner); positive everywhere iff no cell is folded at a corner."""
    d = mesh.shape[0]
    if d == 1:
        return float(np.min(np.diff(mesh[0])))
    if d == 2:
        x, y = mesh[0], mesh[1]
        x00, x10, x11, x01 = x[:-1, :-1], x[1:, :-1], x[1:, 1:], x[:-1, 1:]
        y00, y10, y11, y01 = y[:-1, :-1], y[1:, :-1], y[1:, 1:], y[:-1, 1:]
        area = 0.5 * ((x00 * y10 - x10 * y00) + (x10 * y11 - x11 * y10)
                      + (x11 * y01 - x01 * y11) + (x01 * y00 - x00 * y01))
        return float(np.min(area))
    P = np.moveaxis(mesh, 0, -1)
    best = np.inf
    for c0 in (0, 1):
        for c1 in (0, 1):
            for c2 in (0, 1):
                def corner(o0, o1, o2):
                    return P[o0:P.shape[0] - 1 + o0, o1:P.shape[1] - 1 + o1, o2:P.shape[2] - 1 + o2]
                base = corner(c0, c1, c2)
                e0 = corner(1 - c0, c1, c2) - base
                e1 = corner(c0, 1 - c1, c2) - base
                e2 = corner(c0, c1, 1 - c2) - base
                # orientation: edges point in +axis direction when c = 0, else -axis
                sgn = (1 - 2 * c0) * (1 - 2 * c1) * (1 - 2 * c2)
                J = sgn * np.einsum("...i,...i->...", e0, np.cross(e1, e2))
                best = min(best, float(np.min(J)))
    return best


@dataclass
class Result:
    psi: np.ndarray            # glued Psi on the global grid
    mesh: np.ndarray           # [d, *n]
    res_hist: list             # residual per step (max over subdomains)
    steps: int
    min_det: float
    min_cell: float
    sub_psi: list = None       # per-subdomain Psi (DD)


def solve_single(grid: GridSpec, mon: dict, dt: float, gamma: float, steps: int, tol: float = 0.0,
                 psi0=None, theta_val=None) -> Result:
    """PMA on the whole domain (Sec. 2)."""
    box = grid.whole_box()
    th = theta(mon, grid.lo, grid.hi) if theta_val is None else theta_val
    psi = initial_psi(box) if psi0 is None else np.array(psi0, dtype=np.float64)
    hist = []
    n = 0
    for n in range(1, steps + 1):
        psi, r = step_box(psi, box, mon, th, grid.vol, dt, gamma)
        hist.append(r)
        if tol > 0.0 and r <= tol:
            break
    mesh = mesh_from_psi(psi, box)
    return Result(psi, mesh, hist, n, min_det_hessian(psi, box), min_cell_measure(mesh))


def sweep_order(dec: Decomposition, mode: str) -> list:
    """Order in which the alternating form (Algorithm 1) visits the subdomains."""
    M = len(dec.subs)
    if mode == "alternating":
        return list(range(M))
    if mode == "coloured":
        return sorted(range(M), key=lambda si: (tuple(i % 2 for i in dec.subs[si].index), si))
    raise ValueError(mode)


def solve_dd(grid: GridSpec, parts, overlap_cells, mon: dict, dt: float, gamma: float, steps: int,
             tol: float = 0.0, mode: str = "parallel", stop: str = "max", psi0=None, theta_val=None,
             refresh: bool = True) -> Result:
    """Overlapping DD-PMA.  mode="parallel": eq. transmission_condition3, every subdomain reads
    its neighbours' time-n values.  mode="alternating" / "coloured": Algorithm 1, subdomains swept
    in the order of sweep_order, each reading the latest values.  Glue (Sec. 4.5, "combining"
    the subdomain meshes): refresh the artificial nodes, then take each global node from its
    owner."""
    dec = Decomposition(grid, parts, overlap_cells)
    th = theta(mon, grid.lo, grid.hi) if theta_val is None else theta_val
    if psi0 is None:
        states = [initial_psi(s.box) for s in dec.subs]
    else:
        psi0 = np.asarray(psi0, dtype=np.float64)
        states = []
        for s in dec.subs:
            sl = tuple(slice(s.box.off[k], s.box.off[k] + s.box.n[k]) for k in range(grid.d))
            states.append(psi0[sl].copy())
    hist = []
    n = 0
    for n in range(1, steps + 1):
        res = []
        if mode == "parallel":
            dec.transmit(states)
            new = []
            for si, s in enumerate(dec.subs):
                p, r = step_box(states[si], s.box, mon, th, grid.vol, dt, gamma)
                new.append(p)
                res.append(r)
            states = new
        elif mode in ("alternating", "coloured"):
            for si in sweep_order(dec, mode):
                s = dec.subs[si]
                for o, dst, src in dec.trans[si]:
                    states[si].reshape(-1)[dst] = states[o].reshape(-1)[src]
                states[si], r = step_box(states[si], s.box, mon, th, grid.vol, dt, gamma)
                res.append(r)
        else:
            raise ValueError(mode)
        r = max(res) if stop == "max" else min(res)
        hist.append(r)
        if tol > 0.0 and r <= tol:
            break
    if refresh:
        dec.transmit(states)
    meshes = [mesh_from_psi(states[si], s.box) for si, s in enumerate(dec.subs)]
    mesh = np.stack([dec.glue([m[k] for m in meshes]) for k in range(grid.d)], axis=0)
    psi = dec.glue(states)
    dets = []
    own_dets = []
    for si, s in enumerate(dec.subs):
        _, hess = derivatives(states[si], s.box)
        dets.append(det_sym(hess, grid.d))
    glued_det = dec.glue(dets)
    return Result(psi, mesh, hist, n, float(np.min(glued_det)), min_cell_measure(mesh),
                  sub_psi=states)


# ----------------------------------------------------------------------------------------
# One-dimensional special case and exact equidistribution (used to pin separable monitors).
# ----------------------------------------------------------------------------------------

def equidistribution_exact_sech2(xi: np.ndarray, a: float, b: float, A: float, k: float, c: float):
    """Exact 1D equidistributed map X(xi) for rho_1 = 1 + A sech^2(k (x - c)) on [a, b]:
    int_a^X rho_1 = (xi - a)/(b - a) int_a^b rho_1 (eq. edp in 1D), solved by bracketing on the
    antiderivative R(x) = x + (A/k) tanh(k (x - c))."""
    R = lambda x: x + (A / k) * math.tanh(k * (x - c))
    total = R(b) - R(a)
    out = np.empty_like(xi)
    for i, s in enumerate(xi):
        target = R(a) + total * (s - a) / (b - a)
        if s <= a:
            out[i] = a
        elif s >= b:
            out[i] = b
        else:
            out[i] = scipy.optimize.brentq(lambda x: R(x) - target, a, b, xtol=1e-15, rtol=1e-15)
    return out


# ----------------------------------------------------------------------------------------
# Error and quality measures (Sec. 4.4 eqs. rel_errlp / rel_errlinf; Sec. 4.5).
# ----------------------------------------------------------------------------------------

def rel_errors(ref: np.ndarray, approx: np.ndarray, h) -> dict:
    """E_1, E_2 (trapezoid rule for the integrals) and E_inf."""
    d = ref.ndim
    w = np.ones(ref.shape)
    for k in range(d):
        wk = np.ones(ref.shape[k])
        wk[0] = wk[-1] = 0.5
        shape = [1] * d
        shape[k] = -1
        w = w * wk.reshape(shape)
    w = w * float(np.prod(h))
    diff = np.abs(ref - approx)
    out = {}
    for p in (1, 2):
        out[p] = (np.sum(w * diff ** p) ** (1.0 / p)) / (np.sum(w * np.abs(ref) ** p) ** (1.0 / p))
    out["inf"] = float(np.max(diff) / np.max(np.abs(ref)))
    return out


def quality(psi: np.ndarray, grid: GridSpec, mon: dict, theta_val=None) -> dict:
    """Quality of the mesh x = grad_h Psi (see quality_of_mesh)."""
    return quality_of_mesh(mesh_from_psi(psi, grid.whole_box()), grid, mon, theta_val)


def quality_of_mesh(mesh: np.ndarray, grid: GridSpec, mon: dict, theta_val=None) -> dict:
    """E_adp = |Omega_c| (rho / theta) J at every node (eq. quality_measure with rho
    normalised), J the Jacobian of the mesh x[d, *n] by second-order finite differences of x
    (one-sided at the boundary).  Returns E_2 (trapezoid L2 over Omega_c / |Omega_c|) and
    E_max."""
    box = grid.whole_box()
    th = theta(mon, grid.lo, grid.hi) if theta_val is None else theta_val
    d = grid.d
    Jm = np.empty((d, d) + tuple(grid.n))
    for i in range(d):
        for k in range(d):
            Jm[i, k] = np.gradient(mesh[i], grid.h[k], axis=k, edge_order=2)
    J = det_sym([[Jm[i, k] for k in range(d)] for i in range(d)], d) if d < 3 else np.linalg.det(
        np.moveaxis(Jm, (0, 1), (-2, -1)))
    X = np.moveaxis(mesh, 0, -1)
    E = grid.vol * rho(mon, X) / th * J
    w = box.trapezoid_weights()
    return {"E2": float(math.sqrt(np.sum(w * E * E) / grid.vol)), "Emax": float(np.max(E))}
