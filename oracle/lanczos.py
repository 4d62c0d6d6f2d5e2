"""Stochastic Lanczos quadrature (SLQ) for log det K.

Test infrastructure only (see ``oracle/__init__``).

Sec. 3.3 notes that stochastic trace estimation can replace its circulant
log-determinant; this is that route: log det K = tr log K ~ (1/N) sum_z
z^T log(K) z over probe vectors z, each quadratic form approximated by
Gauss quadrature from m Lanczos steps started at z / ||z||:

    T_m = tridiag(beta, alpha, beta),  eig(T_m) = (theta_i, tau_i),
    z^T log(K) z ~ ||z||^2 sum_i tau_i[0]^2 log theta_i.

The Lanczos recurrence (three-term, optional full reorthogonalisation):
    w = K q_j;  alpha_j = q_j^T w;  r = w - alpha_j q_j - beta_{j-1} q_{j-1};
    beta_j = ||r||;  q_{j+1} = r / beta_j.
An exact zero beta_j (invariant subspace) ends the recurrence early; the
quadrature is then exact for that probe.
"""
import numpy as np
from scipy.linalg import eigh_tridiagonal


def lanczos(matvec, z, m, reorth=True, breakdown_tol=1e-12):
    """Run up to m Lanczos steps from z/||z||; returns (alpha, beta) with
    len(beta) == len(alpha) - 1 (off-diagonals of T)."""
    q = np.asarray(z, dtype=np.float64) / np.linalg.norm(z)
    Q = [q]
    alpha, beta = [], []
    q_prev = np.zeros_like(q)
    b_prev = 0.0
    for j in range(m):
        w = matvec(q)
        a = float(q @ w)
        alpha.append(a)
        r = w - a * q - b_prev * q_prev
        if reorth:
            Qm = np.array(Q).T
            for _ in range(2):
                r = r - Qm @ (Qm.T @ r)
        b = float(np.linalg.norm(r))
        if j == m - 1:
            break
        if b <= breakdown_tol * max(abs(a), b_prev, 1e-300):
            break
        beta.append(b)
        q_prev, q = q, r / b
        b_prev = b
        Q.append(q)
    return np.array(alpha), np.array(beta)


def quadrature(alpha, beta, znorm2):
    """Gauss quadrature of z^T log(K) z from the Lanczos coefficients."""
    if len(alpha) == 1:
        return znorm2 * np.log(alpha[0])
    th, V = eigh_tridiagonal(alpha, beta)
    return znorm2 * float(np.sum(V[0, :] ** 2 * np.log(th)))


def combine(vals, coloured):
    """Estimate and standard error from per-probe quadratic forms.

    Rademacher probes satisfy E[z z^T] = I, so the estimate is the mean over
    probes and the standard error is std / sqrt(N).  Coloured probes satisfy
    E[sum_k z_k z_k^T] = I, so the estimate is the sum; its spread is
    reported as sqrt(N) * std (treating the colour classes as exchangeable).
    """
    vals = np.asarray(vals, dtype=np.float64)
    N = len(vals)
    sd = float(np.std(vals, ddof=1)) if N > 1 else 0.0
    if coloured:
        return float(vals.sum()), float(np.sqrt(N) * sd)
    return float(vals.mean()), sd / np.sqrt(N)


def slq_logdet(matvec, probes, m, reorth=True, coloured=False):
    """SLQ estimate of log det K with the given probes (p, N).

    Returns (estimate, standard error, per-probe values, steps per probe).
    Probes that are identically zero contribute 0.
    """
    probes = np.asarray(probes, dtype=np.float64)
    vals, steps = [], []
    for k in range(probes.shape[1]):
        z = probes[:, k]
        zz = float(z @ z)
        if zz == 0.0:
            vals.append(0.0)
            steps.append(0)
            continue
        a, b = lanczos(matvec, z, m, reorth=reorth)
        vals.append(quadrature(a, b, zz))
        steps.append(len(a))
    est, se = combine(vals, coloured)
    return est, se, np.array(vals), np.array(steps)


def check_steps(longest, every=5):
    """Step counts at which the adaptive mode checks: every, 2 every, ...,
    then each check `every` * max(1, floor(j / 50)) steps after the last
    (every 5 steps up to 100, every 10 up to 150, every 15 up to 200, ...)."""
    out, j = [], every
    while j <= longest:
        out.append(j)
        j += every * max(1, j // 50)
    return out


def adaptive_steps(alphas, betas, znorm2s, rtol, every=5, first=10):
    """Step count at which the adaptive mode stops: at each check of
    `check_steps` from `first` on, every probe's quadrature value with the
    steps so far must have moved by at most rtol times its size since the
    previous check; otherwise (including when every recurrence ended before
    the first check) all the steps that were run.  A probe whose recurrence
    ended earlier keeps its final value (it no longer moves).  This stopping
    rule is the library's own (the paper fixes the step count).
    alphas / betas: per-probe coefficient arrays of the full run."""
    longest = max((len(a) for a in alphas), default=0)

    def gammas(j):
        out = []
        for a, b, zz in zip(alphas, betas, znorm2s):
            if zz == 0.0 or len(a) == 0:
                out.append(0.0)
                continue
            s = min(j, len(a))
            out.append(quadrature(a[:s], b[: s - 1], zz))
        return np.array(out)

    prev = None
    for j in check_steps(longest, every):
        cur = gammas(j)
        if j >= first and prev is not None and np.all(np.abs(cur - prev) <= rtol * np.abs(cur)):
            return j
        prev = cur
    return longest


def slq_logdet_adaptive(matvec, probes, max_steps, rtol, reorth=True, coloured=False):
    """SLQ with the adaptive stopping rule of `adaptive_steps` (Lanczos run
    to max_steps, then cut where the rule stops; the coefficients of the first
    j steps do not depend on later ones).  Returns (estimate, standard error,
    per-probe values, steps used)."""
    probes = np.asarray(probes, dtype=np.float64)
    alphas, betas, zzs = [], [], []
    for k in range(probes.shape[1]):
        z = probes[:, k]
        zz = float(z @ z)
        zzs.append(zz)
        if zz == 0.0:
            alphas.append(np.zeros(0))
            betas.append(np.zeros(0))
            continue
        a, b = lanczos(matvec, z, max_steps, reorth=reorth)
        alphas.append(a)
        betas.append(b)
    m = adaptive_steps(alphas, betas, zzs, rtol)
    vals = []
    for a, b, zz in zip(alphas, betas, zzs):
        if zz == 0.0:
            vals.append(0.0)
            continue
        s = min(m, len(a))
        vals.append(quadrature(a[:s], b[: s - 1], zz))
    est, se = combine(vals, coloured)
    return est, se, np.array(vals), m


def exact_hutchinson(K, probes, coloured=False):
    """The probe estimate with every z^T log(K) z computed exactly from a dense
    eigendecomposition (separates probe error from quadrature error)."""
    w, V = np.linalg.eigh(K)
    P = V.T @ np.asarray(probes, dtype=np.float64)
    per = np.sum(P * P * np.log(w)[:, None], axis=0)
    return combine(per, coloured)[0], per
