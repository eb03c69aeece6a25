"""Independent numpy formulations used to pin the oracle (test helpers only).

- `qz`, `charmatrix`: the characteristic-matrix (Abeles / Heavens) thin-film
  solve, converted to the amplitude convention of Eq. 3.
- `maxwell_event`: a plane wave meeting a planar multilayer, solved directly
  from Maxwell's boundary conditions in laboratory coordinates: every wave's
  field is an unknown complex 3-vector constrained to be transverse to its
  (complex) wave vector, and the tangential E and H are continuous at every
  interface.  No s/p decomposition, Fresnel formula or sign convention
  enters; the reflected and transmitted field vectors come out of one linear
  solve.  It therefore checks, at once, the interface coefficients (Eq. 3),
  the multilayer response (Eq. 4 and the transfer-matrix method) and the
  polarization bookkeeping of Eq. 5 (which component is multiplied by which
  coefficient, and on which outgoing basis).

Time dependence exp(-i w t): a wave exp(i k . r) with Im(k . u) >= 0 decays
along the direction of travel u, which fixes the evanescent branch.
"""
import numpy as np


def qz(N, kappa):
    """Normal wavenumber sqrt(N^2 - kappa^2) on the branch Im q >= 0 (Re q >= 0 when real)."""
    q = np.sqrt(np.complex128(N) ** 2 - kappa ** 2)
    if q.imag < 0 or (q.imag == 0 and q.real < 0):
        q = -q
    return q


def charmatrix(thk, N, n0, ns, lam, kappa):
    """Characteristic-matrix solve (exp(-i w t)), converted to Eq. 3 amplitudes."""
    k0 = 2 * np.pi / lam
    q0, qs = qz(n0, kappa), qz(ns, kappa)
    out = []
    for pol in (0, 1):
        eta0 = q0 if pol == 0 else n0 ** 2 / q0
        etas = qs if pol == 0 else ns ** 2 / qs
        Mt = np.eye(2, dtype=np.complex128)
        for d, n in zip(thk, N):
            q = qz(n, kappa)
            eta = q if pol == 0 else n ** 2 / q
            dl = k0 * q * d
            Mj = np.array([[np.cos(dl), -1j * np.sin(dl) / eta], [-1j * eta * np.sin(dl), np.cos(dl)]])
            Mt = Mt @ Mj
        B, Cc = Mt @ np.array([1.0, etas])
        r = (eta0 * B - Cc) / (eta0 * B + Cc)
        t = 2 * eta0 / (eta0 * B + Cc)
        if pol == 1:
            r = -r
            t = t * (q0 / n0) / (qs / ns)
        out.append((r, t))
    (rs, ts), (rp, tp) = out
    return np.array([rs, rp, ts, tp])


def _tangents(u):
    a = np.array([1.0, 0.0, 0.0]) if abs(u[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    t1 = a - (a @ u) * u
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(u, t1)
    return t1, t2


def maxwell_event(d, E0, u, n0, layers, n_out, lam_nm):
    """Plane wave in a lossless medium of index n0 with real unit direction d
    and complex field E0 (transverse to d) meets planar layers stacked along
    the unit normal u (d . u > 0).  `layers` lists (N_j, thickness_nm) in the
    order met; n_out is the exit medium.

    Returns (E_r, k_r, E_t, k_t): the reflected field at the first interface
    and the transmitted field at the last one, with their wave vectors in
    units of the vacuum wavenumber (k . k = N^2; k_t is complex for an
    evanescent exit wave).  Phases of waves inside layer j are referenced at
    the interface each wave enters from, so every exponential has modulus <= 1.
    """
    d = np.asarray(d, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    E0 = np.asarray(E0, dtype=np.complex128)
    k0 = 2.0 * np.pi / lam_nm
    kt = n0 * (d - (d @ u) * u)            # conserved tangential wave vector
    kap = float(np.linalg.norm(kt))
    media = [complex(n0)] + [complex(N) for N, _ in layers] + [complex(n_out)]
    thk = [0.0] + [float(t) for _, t in layers] + [0.0]
    q = [qz(N, kap) for N in media]
    L = len(layers)
    k_in = n0 * d
    # unknown waves: (medium, direction sign); incident medium: reflected only;
    # layers: forward and backward; exit: forward only
    waves = [(0, -1)] + [(j, s) for j in range(1, L + 1) for s in (+1, -1)] + [(L + 1, +1)]
    col = {w: 3 * i for i, w in enumerate(waves)}
    n_unk = 3 * len(waves)
    kvec = {w: kt + w[1] * q[w[0]] * u for w in waves}
    A = np.zeros((n_unk, n_unk), dtype=np.complex128)
    b = np.zeros(n_unk, dtype=np.complex128)
    row = 0
    for w in waves:                          # transversality k . E = 0 (bilinear)
        A[row, col[w]:col[w] + 3] = kvec[w]
        row += 1
    t1, t2 = _tangents(u)

    def phase(w, at_interface):
        j, s = w
        if j == 0 or j == L + 1:
            return 1.0
        # forward waves referenced at interface j-1 (entrance), backward at j
        far = (s > 0 and at_interface == j) or (s < 0 and at_interface == j - 1)
        return np.exp(1j * k0 * q[j] * thk[j]) if far else 1.0

    def cross_mat(k):
        return np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]], dtype=np.complex128)

    for i in range(L + 1):                   # interface between media i and i + 1
        left = [w for w in waves if w[0] == i]
        right = [w for w in waves if w[0] == i + 1]
        for t in (t1, t2):
            # tangential E: sum_left - sum_right = -(incident, if i == 0)
            for w in left:
                A[row, col[w]:col[w] + 3] += phase(w, i) * t
            for w in right:
                A[row, col[w]:col[w] + 3] -= phase(w, i) * t
            if i == 0:
                b[row] -= t @ E0
            row += 1
            # tangential H = k x E
            for w in left:
                A[row, col[w]:col[w] + 3] += phase(w, i) * (t @ cross_mat(kvec[w]))
            for w in right:
                A[row, col[w]:col[w] + 3] -= phase(w, i) * (t @ cross_mat(kvec[w]))
            if i == 0:
                b[row] -= t @ np.cross(k_in, E0)
            row += 1
    assert row == n_unk
    X = np.linalg.solve(A, b)
    r_w, t_w = waves[0], waves[-1]
    return X[col[r_w]:col[r_w] + 3], kvec[r_w], X[col[t_w]:col[t_w] + 3], kvec[t_w]


def normal_flux(E, k, u):
    """Time-averaged power flux of a plane wave across a plane of normal u,
    Re(E x conj(k x E)) . u, in the units of `maxwell_event` (nonmagnetic)."""
    H = np.cross(k, E)
    return float(np.real(np.cross(E, np.conj(H))) @ u)
