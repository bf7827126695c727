"""Closed-form results for uniform and cycloidal states of the spin
Hamiltonian (Methods, Eq. param-hamiltonian) on the periodic rhombic
triangular lattice.  Written from the mathematics, independently of the
oracle, so that they can pin it.

Lattice: a1 = (1, 0), a2 = (1/2, sqrt3/2); reciprocal vectors
b1 = 2pi (1, -1/sqrt3), b2 = 2pi (0, 2/sqrt3); allowed wave vectors of an
Lx x Ly periodic cell: k = n1 b1 / Lx + n2 b2 / Ly.
Shell s of the triangular lattice: the 6 (or 12) lattice vectors at the s-th
distance; the first three are listed explicitly below.
"""
import numpy as np

SQ3 = np.sqrt(3.0)
A1 = np.array([1.0, 0.0])
A2 = np.array([0.5, SQ3 / 2])
B1 = 2 * np.pi * np.array([1.0, -1.0 / SQ3])
B2 = 2 * np.pi * np.array([0.0, 2.0 / SQ3])

# the three nearest shells as lattice offsets (independent listing)
SHELL_OFFSETS = [
    [(1, 0), (0, 1), (-1, 1), (-1, 0), (0, -1), (1, -1)],
    [(1, 1), (-1, 2), (-2, 1), (-1, -1), (1, -2), (2, -1)],
    [(2, 0), (0, 2), (-2, 2), (-2, 0), (0, -2), (2, -2)],
]


def _table_s1_offsets():
    """Offsets of all 35 shells, enumerated from the distances and bond counts
    of the paper's Table S1 (tests/golden fixture; distances in units of the
    lattice constant a, nearest neighbour a/sqrt2): shell s holds every
    lattice vector whose squared length, in nearest-neighbour units, is the
    s-th printed distance squared.  The three hand-listed shells come first."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table_s1_shells.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    out = []
    for r, cnt in rows:
        d2 = int(round((float(r) / 0.707107) ** 2))
        offs = [(dx, dy) for dy in range(-12, 13) for dx in range(-12, 13) if dx * dx + dx * dy + dy * dy == d2]
        assert len(offs) == int(cnt), (r, cnt, len(offs))
        out.append(offs)
    for s in range(3):
        assert sorted(out[s]) == sorted(SHELL_OFFSETS[s])
    return out


SHELL_OFFSETS_35 = _table_s1_offsets()


def shell_count(s):
    return len(SHELL_OFFSETS_35[s])


def cart(dx, dy):
    return dx * A1 + dy * A2


def kgrid(Lx, Ly):
    n1, n2 = np.meshgrid(np.arange(Lx), np.arange(Ly), indexing="ij")
    k = (n1[..., None] * B1 / Lx + n2[..., None] * B2 / Ly).reshape(-1, 2)
    return k


def shell_sum(k, s):
    """S_s(k) = sum_{delta in shell s} (1 - cos k.delta)."""
    out = np.zeros(len(k))
    for dx, dy in SHELL_OFFSETS_35[s]:
        d = cart(dx, dy)
        out += 1.0 - np.cos(k @ d)
    return out


def dmi_sine_sum(k):
    """S_D(k) = sum_{delta in NN} dhat_y sin(k.delta)."""
    out = np.zeros(len(k))
    for dx, dy in SHELL_OFFSETS[0]:
        d = cart(dx, dy)
        out += d[1] * np.sin(k @ d)
    return out


def fm_z_spectrum(Lx, Ly, J, K, bz):
    """All 2N tangent-Hessian eigenvalues of the uniform state m = +z with
    B = bz z: lambda(k) = 2 sum_s J_s S_s(k) + bz + 2K, twice for every k
    (the two transverse polarisations decouple; interfacial DMI drops out)."""
    k = kgrid(Lx, Ly)
    lam = np.full(len(k), bz + 2 * K)
    for s, Js in enumerate(J):
        lam = lam + 2 * Js * shell_sum(k, s)
    return np.sort(np.concatenate([lam, lam]))


def fm_z_energy(N, J, K, bz):
    """E/N = -sum_delta J_delta - bz - K for m = +z (every offset of every
    shell: 6, 12 or 24 per shell)."""
    return N * (-sum(shell_count(s) * Js for s, Js in enumerate(J)) - bz - K)


def fm_x_spectrum(Lx, Ly, J, D1, K, bx):
    """All 2N eigenvalues at the uniform state m = +x with B = bx x, easy
    axis z and NN interfacial DMI D1:
      lambda_pm(k) = 2 sum_s J_s S_s(k) + bx - K +- sqrt(K^2 + 4 D1^2 S_D(k)^2)."""
    k = kgrid(Lx, Ly)
    base = bx - K
    for s, Js in enumerate(J):
        base = base + 2 * Js * shell_sum(k, s)
    rad = np.sqrt(K * K + 4 * D1 * D1 * dmi_sine_sum(k) ** 2)
    return np.sort(np.concatenate([base - rad, base + rad]))


def cycloid_state(Lx, Ly, n1, n2):
    """Commensurate Neel cycloid m(r) = cos(q.r) z + sin(q.r) qhat with
    q = n1 b1/Lx + n2 b2/Ly."""
    q = n1 * B1 / Lx + n2 * B2 / Ly
    qh = q / np.linalg.norm(q)
    y, x = np.divmod(np.arange(Lx * Ly), Lx)
    r = x[:, None] * A1 + y[:, None] * A2
    ph = r @ q
    m = np.stack([np.sin(ph) * qh[0], np.sin(ph) * qh[1], np.cos(ph)])
    return m, q, ph


def cycloid_energy(Lx, Ly, n1, n2, J, D1, K, bz):
    """E = N[-sum_delta J_delta cos(q.delta) - D1 sum_{delta in NN}
    (dhat.qhat) sin(q.delta)] - K sum_i cos^2(q.r_i) - bz sum_i cos(q.r_i)."""
    m, q, ph = cycloid_state(Lx, Ly, n1, n2)
    N = Lx * Ly
    qh = q / np.linalg.norm(q)
    e = 0.0
    for s, Js in enumerate(J):
        for dx, dy in SHELL_OFFSETS_35[s]:
            e += -Js * np.cos(q @ cart(dx, dy))
    for dx, dy in SHELL_OFFSETS[0]:
        d = cart(dx, dy)
        e += -D1 * (d @ qh) * np.sin(q @ d)
    return N * e - K * np.sum(np.cos(ph) ** 2) - bz * np.sum(np.cos(ph))


def sw_minima(bx, K):
    """Uniform minima (h, 0, +-sqrt(1 - h^2)), h = bx / (2K), for D = 0."""
    h = bx / (2 * K)
    return np.array([h, 0.0, np.sqrt(1 - h * h)]), np.array([h, 0.0, -np.sqrt(1 - h * h)])


def sw_barrier(N, bx, K):
    """Coherent-rotation barrier E(x) - E(min) = N K (1 - h)^2."""
    h = bx / (2 * K)
    return N * K * (1 - h) ** 2
