"""Plain FP64 reference implementation of one MRA alignment pass.

TEST INFRASTRUCTURE, NOT PRODUCT CODE (see the package docstring).  Every
function takes the exact float32 arrays handed to the GPU, promotes them to
float64 and evaluates the paper's definitions directly:

* Sec. 2: the rotational cross-correlation between a particle x and a
  reference y is the integral, over radii r1..r2 and over the full circle, of
  x(r, theta) * y(r, theta + phi) * |r|.  Discretised here on integer rings
  r = r_min..r_max with weight w_r = r and n_phi uniform angles per ring; the
  d(theta) dr constants are dropped.
* Sec. 2 / Sec. 3 (re-sample to polar coordinates, RPC): every particle is
  resampled on the polar grid once per integer shift of the search range, and
  also in mirrored form (the CC table holds "all (mirrored) images").
* Algorithm 1: the best CC over every reference, shift, angle and mirror is
  kept per particle (the reduction of Fig. 2), the alignment parameters are
  decoded from its index, and new class averages are computed from the
  aligned images.

Readings of points the paper leaves open (centre, axes, interpolation, edge,
normalisation, lag direction, tie rule, mirror axis) are fixed in
``Geometry`` and in the docstrings below.

Nothing here uses an FFT: the CC is the direct sum over rings and angles.  The
only library primitive is a float64 matrix product that evaluates many of
those direct sums at once (``cc_table``).
"""

from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class Geometry:
    """Sampling geometry of one alignment problem.

    L          box size in pixels (square images, row-major, x = column,
               y = row, pixel centres at integer coordinates).
    r_min,r_max  first and last integer ring radius (inclusive).
    n_phi      angles per ring; theta_j = 2*pi*j/n_phi measured from +x
               towards +y.
    shift_max  T: integer shifts s in {-T..T}^2 are searched.
    mirror     1: both mirrors are searched, 0: only the unmirrored image.
    normalize  1: every reference is divided by its weighted ring norm.
    """

    L: int
    r_min: int
    r_max: int
    n_phi: int
    shift_max: int
    mirror: int = 1
    normalize: int = 1

    @property
    def n_rings(self) -> int:
        return self.r_max - self.r_min + 1

    @property
    def n_mirror(self) -> int:
        return 2 if self.mirror else 1

    @property
    def n_shift_axis(self) -> int:
        return 2 * self.shift_max + 1


def centre(L: int) -> tuple[int, int]:
    """Sampling centre (c_x, c_y) = (floor(L/2), floor(L/2))."""
    return L // 2, L // 2


def ring_radii(g: Geometry) -> np.ndarray:
    return np.arange(g.r_min, g.r_max + 1, dtype=np.float64)


def ring_weights(g: Geometry) -> np.ndarray:
    """The |r| factor of the Sec. 2 correlation integral: w_r = r."""
    return ring_radii(g).copy()


def bilinear(img: np.ndarray, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Bilinear interpolation of ``img`` at (x, y); the image is zero outside
    the box [0, L-1]^2 (each of the four neighbours outside contributes 0)."""
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    x0 = np.floor(x)
    y0 = np.floor(y)
    fx = x - x0
    fy = y - y0
    x0 = x0.astype(np.int64)
    y0 = y0.astype(np.int64)

    def pix(ix, iy):
        inside = (ix >= 0) & (ix < W) & (iy >= 0) & (iy < H)
        v = np.zeros(np.broadcast(ix, iy).shape, dtype=np.float64)
        v[inside] = img[iy[inside], ix[inside]]
        return v

    return ((1.0 - fx) * (1.0 - fy) * pix(x0, y0)
            + fx * (1.0 - fy) * pix(x0 + 1, y0)
            + (1.0 - fx) * fy * pix(x0, y0 + 1)
            + fx * fy * pix(x0 + 1, y0 + 1))


def polar_positions(g: Geometry, sx: int, sy: int, m: int):
    """Sample positions of the polar grid for shift (sx, sy) and mirror m.

    x = c_x + sx + r cos(theta_j),  y = c_y + sy + (1 - 2m) r sin(theta_j).
    The mirror flips the image about the horizontal line through the
    sampling centre, so mirrored samples are taken at negated angles.
    Returns two arrays of shape [n_rings, n_phi].
    """
    cx, cy = centre(g.L)
    r = ring_radii(g)[:, None]
    th = 2.0 * np.pi * np.arange(g.n_phi, dtype=np.float64)[None, :] / g.n_phi
    x = cx + sx + r * np.cos(th)
    y = cy + sy + (1 - 2 * m) * r * np.sin(th)
    return x, y


def polar_samples(img: np.ndarray, g: Geometry, sx: int = 0, sy: int = 0,
                  m: int = 0) -> np.ndarray:
    """Polar resampling (RPC) of one image: p[r][j], shape [n_rings, n_phi]."""
    x, y = polar_positions(g, sx, sy, m)
    return bilinear(img, x, y)


def particle_polar(img: np.ndarray, g: Geometry) -> np.ndarray:
    """All shifted and mirrored polar images of one particle.

    Shape [M, 2T+1 (sy), 2T+1 (sx), n_rings, n_phi]; the mirror is resampled
    directly at mirrored positions, never derived from the unmirrored samples.
    """
    T = g.shift_max
    out = np.empty((g.n_mirror, g.n_shift_axis, g.n_shift_axis, g.n_rings, g.n_phi))
    for m in range(g.n_mirror):
        for iy, sy in enumerate(range(-T, T + 1)):
            for ix, sx in enumerate(range(-T, T + 1)):
                out[m, iy, ix] = polar_samples(img, g, sx, sy, m)
    return out


def reference_polar(refs: np.ndarray, g: Geometry):
    """Polar samples of every reference at zero shift, unmirrored.

    Returns (qhat [K, n_rings, n_phi], nu [K]) with nu_k the weighted ring
    norm sqrt(sum_r w_r sum_j q^2); qhat = q / nu when ``g.normalize`` else q.
    A zero-norm reference with normalisation on raises ValueError.
    """
    refs = np.asarray(refs, dtype=np.float64)
    w = ring_weights(g)
    q = np.stack([polar_samples(refs[k], g) for k in range(refs.shape[0])])
    nu = np.sqrt(np.einsum("r,krj->k", w, q * q))
    if g.normalize:
        if np.any(nu == 0.0):
            raise ValueError("reference with zero weighted ring norm")
        q = q / nu[:, None, None]
    return q, nu


def rolled_reference_matrix(qhat: np.ndarray, g: Geometry) -> np.ndarray:
    """Matrix B with B[(r, j), (k, a)] = w_r * qhat_k[r][(j + a) mod n_phi].

    A row of particle samples p[(r, j)] times B gives, for every reference k
    and lag a, the direct sum  sum_r w_r sum_j p[r][j] qhat_k[r][(j+a)].
    """
    K, R, n = qhat.shape
    j = np.arange(n)[:, None]
    a = np.arange(n)[None, :]
    idx = (j + a) % n                                      # [j, a]
    rolled = qhat[:, :, idx]                               # [K, R, j, a]
    rolled = rolled * ring_weights(g)[None, :, None, None]
    return np.ascontiguousarray(rolled.transpose(1, 2, 0, 3).reshape(R * n, K * n))


def cc_table(parts: np.ndarray, refs: np.ndarray, g: Geometry,
             qhat: np.ndarray | None = None,
             bmat: np.ndarray | None = None) -> np.ndarray:
    """Full CC table C[n, k, m, sy+T, sx+T, a] by direct ring sums.

    C[n,k,s,m,a] = sum_r w_r sum_j p_{n,s,m}[r][j] * qhat_k[r][(j + a) mod n_phi]
    (Sec. 2 correlation; the particle is the unshifted-angle operand and the
    reference is read at theta_j + phi_a).
    """
    parts = np.asarray(parts, dtype=np.float64)
    if qhat is None:
        qhat, _ = reference_polar(refs, g)
    if bmat is None:
        bmat = rolled_reference_matrix(qhat, g)
    K = qhat.shape[0]
    n = g.n_phi
    S = g.n_shift_axis
    M = g.n_mirror
    out = np.empty((parts.shape[0], K, M, S, S, n))
    for i in range(parts.shape[0]):
        p = particle_polar(parts[i], g).reshape(M * S * S, g.n_rings * n)
        c = (p @ bmat).reshape(M, S, S, K, n)
        out[i] = c.transpose(3, 0, 1, 2, 4)
    return out


def flat_index(g: Geometry, k, m, sx, sy, a):
    """Candidate index used for the tie rule: the smallest index wins.

    iota = (((k*M + m)*(2T+1) + (sy+T))*(2T+1) + (sx+T))*n_phi + a
    """
    T = g.shift_max
    S = g.n_shift_axis
    return ((((np.asarray(k) * g.n_mirror + m) * S + (np.asarray(sy) + T)) * S
             + (np.asarray(sx) + T)) * g.n_phi + a)


def _decode(g: Geometry, iota: int):
    T = g.shift_max
    S = g.n_shift_axis
    a = iota % g.n_phi
    rest = iota // g.n_phi
    sx = rest % S - T
    rest //= S
    sy = rest % S - T
    rest //= S
    m = rest % g.n_mirror
    k = rest // g.n_mirror
    return int(k), int(m), int(sx), int(sy), int(a)


def align(parts: np.ndarray, refs: np.ndarray, g: Geometry, batch: int = 8) -> dict:
    """Best alignment of every particle (Algorithm 1, arg-max of Fig. 2).

    The winner maximises C over (k, m, s, a); among exactly equal values the
    smallest ``flat_index`` wins.  ``cc2`` is the best value over every other
    candidate (including the neighbouring angles of the winner).  The reported
    in-plane angle is psi = (n_phi - a) mod n_phi, so that a particle made by
    rotating a reference by psi*2*pi/n_phi is reported with that psi.
    """
    parts = np.asarray(parts, dtype=np.float64)
    N = parts.shape[0]
    qhat, _ = reference_polar(refs, g)
    bmat = rolled_reference_matrix(qhat, g)
    res = {key: np.zeros(N, dtype=np.int64)
           for key in ("ref", "shift_x", "shift_y", "psi", "mirror", "flat_index")}
    res["cc"] = np.zeros(N)
    res["cc2"] = np.zeros(N)
    for lo in range(0, N, batch):
        tab = cc_table(parts[lo:lo + batch], None, g, qhat=qhat, bmat=bmat)
        for i in range(tab.shape[0]):
            flat = tab[i].reshape(-1)          # ordered exactly as flat_index
            iota = int(np.argmax(flat))        # first maximum = smallest index
            best = flat[iota]
            flat[iota] = -np.inf
            k, m, sx, sy, a = _decode(g, iota)
            n = lo + i
            res["ref"][n] = k
            res["mirror"][n] = m
            res["shift_x"][n] = sx
            res["shift_y"][n] = sy
            res["psi"][n] = (g.n_phi - a) % g.n_phi
            res["flat_index"][n] = iota
            res["cc"][n] = best
            res["cc2"][n] = flat.max() if flat.size > 1 else -np.inf
    return res


def candidate_cc(img: np.ndarray, qhat_k: np.ndarray, g: Geometry,
                 sx: int, sy: int, m: int, a: int) -> float:
    """CC of one candidate (k, s, m, a) as a direct double sum."""
    p = polar_samples(img, g, sx, sy, m)
    q = np.roll(np.asarray(qhat_k, dtype=np.float64), -a, axis=1)  # q[(j+a)]
    return float(np.sum(ring_weights(g)[:, None] * p * q))


def averages(parts: np.ndarray, params: dict, prev: np.ndarray, g: Geometry):
    """Class-average update from aligned images (Algorithm 1).

    For each class k with n_k > 0:
      Y'_k(u) = (1/n_k) sum_{n: ref_n = k} Bil(X_n; c + s_n + Mir^{m_n} Rot(alpha_n)(u - c))
    with alpha_n = psi_n * 2*pi/n_phi, Rot(alpha) the counter-clockwise
    rotation in (x, y) and Mir = diag(1, -1).  This inverse warp takes each
    particle back into its reference's frame.  Empty classes keep Y_k.
    Returns (Y' [K, L, L], counts [K]).
    """
    parts = np.asarray(parts, dtype=np.float64)
    prev = np.asarray(prev, dtype=np.float64)
    K, L, _ = prev.shape
    cx, cy = centre(L)
    yy, xx = np.mgrid[0:L, 0:L].astype(np.float64)
    vx = xx - cx
    vy = yy - cy
    sums = np.zeros((K, L, L))
    counts = np.zeros(K, dtype=np.int64)
    for n in range(parts.shape[0]):
        k = int(params["ref"][n])
        alpha = 2.0 * np.pi * float(params["psi"][n]) / g.n_phi
        ca, sa = np.cos(alpha), np.sin(alpha)
        rx = ca * vx - sa * vy
        ry = sa * vx + ca * vy
        if int(params["mirror"][n]):
            ry = -ry
        x = cx + float(params["shift_x"][n]) + rx
        y = cy + float(params["shift_y"][n]) + ry
        sums[k] += bilinear(parts[n], x, y)
        counts[k] += 1
    out = prev.copy()
    for k in range(K):
        if counts[k] > 0:
            out[k] = sums[k] / counts[k]
    return out, counts


def classify(parts: np.ndarray, refs: np.ndarray, g: Geometry, max_iter: int = 20,
             max_changed_frac: float = 0.005):
    """Iterative MRA: the outer loop of Algorithm 1 (align every image against
    the current references, replace the references by the class averages of
    the aligned images, repeat until convergence).

    The paper fixes no convergence rule.  Reading used: stop after a pass in
    which the fraction of particles whose class (ref) differs from the
    previous pass is at most ``max_changed_frac``, or after ``max_iter``
    passes (the test is made on the count: changed <= max_changed_frac * N).
    The averages enter the next pass as float32 images (the type in
    which references are handed to a pass).  Returns (params of the last pass,
    averages after it [K, L, L] float32, counts, passes run, the changed
    fractions of passes 2, 3, ...).
    """
    Y = np.asarray(refs, dtype=np.float32)
    prev = None
    fracs = []
    params, counts, it = None, None, 0
    for it in range(1, max_iter + 1):
        params = align(parts, Y, g)
        Yn, counts = averages(parts, params, Y, g)
        Y = Yn.astype(np.float32)
        if prev is not None:
            n_changed = int(np.count_nonzero(params["ref"] != prev))
            fracs.append(n_changed / len(prev))
            if n_changed <= max_changed_frac * len(prev):
                break
        prev = params["ref"].copy()
    return params, Y, counts, it, fracs


def rfa(parts: np.ndarray, g: Geometry, max_iter: int = 10, max_changed_frac: float = 0.0,
        init: np.ndarray | None = None):
    """Reference-free alignment (RFA, the routine of GPU ISAC that the paper
    builds its MRA on and benchmarks beside it, Sec. 2 and Sec. 5): every
    particle is aligned against one running average, which is then rebuilt
    from the aligned particles, and the two steps repeat.  It is the MRA pass
    and average update with a single reference.

    The paper does not spell the routine out.  Readings used: the first
    reference is the plain mean of the unaligned particles (``init``
    overrides it); every pass searches the whole shift grid around the box
    centre, both mirrors and all angles (no composition with the previous
    parameters, no re-centring of the average); the loop stops after a pass
    in which at most ``max_changed_frac * N`` particles changed any
    parameter (shift, angle or mirror) since the pass before, or after
    ``max_iter`` passes.  Returns (params of the last pass, average after it
    [L, L] float32, passes run, changed fraction of passes 2, 3, ...).
    """
    parts = np.asarray(parts)
    N = parts.shape[0]
    if init is None:
        Y = parts.astype(np.float64).mean(axis=0).astype(np.float32)[None]
    else:
        Y = np.asarray(init, dtype=np.float32).reshape(1, g.L, g.L)
    prev = None
    fracs = []
    params, it = None, 0
    for it in range(1, max_iter + 1):
        params = align(parts, Y, g)
        Y = averages(parts, params, Y, g)[0].astype(np.float32)
        if prev is not None:
            n_changed = int(np.count_nonzero(params["flat_index"] != prev))
            fracs.append(n_changed / N)
            if n_changed <= max_changed_frac * N:
                break
        prev = params["flat_index"].copy()
    return params, Y[0], it, fracs


def refine_psi(parts: np.ndarray, refs: np.ndarray, g: Geometry, params: dict) -> np.ndarray:
    """Sub-step in-plane angle of each particle's winner (an optional
    refinement; the paper searches integer angle steps only).

    A parabola through the CC at the winning lag a and at a - 1, a + 1
    (direct double sums) peaks at a + d with
    d = (c(a-1) - c(a+1)) / (2 (c(a-1) - 2 c(a) + c(a+1))); d = 0 when the
    three values do not curve downwards, and d is clamped to [-1/2, 1/2].
    The refined angle, in steps of 2 pi / n_phi like psi, is (psi - d) mod
    n_phi (psi = -a).
    """
    parts = np.asarray(parts)
    qhat, _ = reference_polar(refs, g)
    out = np.empty(parts.shape[0])
    for n in range(parts.shape[0]):
        k, m = int(params["ref"][n]), int(params["mirror"][n])
        sx, sy, psi = int(params["shift_x"][n]), int(params["shift_y"][n]), int(params["psi"][n])
        a = (g.n_phi - psi) % g.n_phi
        cm, c0, cp = (candidate_cc(parts[n], qhat[k], g, sx, sy, m, (a + d) % g.n_phi) for d in (-1, 0, 1))
        den = cm - 2.0 * c0 + cp
        d = 0.5 * (cm - cp) / den if den < 0.0 else 0.0
        d = min(0.5, max(-0.5, d))
        out[n] = (psi - d) % g.n_phi
    return out
