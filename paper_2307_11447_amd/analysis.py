"""Host analysis of H4D trial logs: the chemical potential from the work
distributions of trial insertions and deletions (Crooks' theorem solved by
Bennett's acceptance ratio, the supplement's section on CFT and BAR), the
acceptance probability predicted from the same distributions (Eq. 21) and
their non-Gaussianity alpha_2.

Work values are the insertion-signed dM of the trial records (dM = dH - I/beta
for an insertion, -dH - I/beta for a deletion, I = 2 ln(V / (Lambda^3
(N+1)))), so that an insertion's ln R is -beta dM + beta mu and a
deletion's beta dM - beta mu.  They come from trials that are never
accepted (the particle numbers stay fixed while they are sampled)."""
import math

import numpy as np


def _fermi(x):
    """1 / (1 + e^x), computed without overflow."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    pos = x > 0
    e = np.exp(-x[pos])
    out[pos] = e / (1.0 + e)
    out[~pos] = 1.0 / (1.0 + np.exp(x[~pos]))
    return out


def bar_beta_mu(dM_ins, dM_del, beta):
    """beta mu from Bennett's acceptance ratio: the root in mu of
    sum_ins f(beta (C + dM - mu)) - sum_del f(-beta (C + dM - mu)),
    f(x) = 1 / (1 + e^x), C = ln(N_ins / N_del) / beta; the insertion sum
    rises and the deletion sum falls with mu, so the root is unique, lies
    within the range of the work values widened by 50 kT, and is found by
    bisection to machine precision."""
    a = np.asarray(dM_ins, dtype=np.float64)
    b = np.asarray(dM_del, dtype=np.float64)
    a, b = a[np.isfinite(a)], b[np.isfinite(b)]
    if len(a) == 0 or len(b) == 0:
        raise ValueError("BAR needs insertion and deletion work values")
    C = math.log(len(a) / len(b)) / beta

    def g(mu):
        return _fermi(beta * (C + a - mu)).sum() - _fermi(-beta * (C + b - mu)).sum()

    lo = min(a.min(), b.min()) - 50.0 / beta
    hi = max(a.max(), b.max()) + 50.0 / beta
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(mid) > 0.0:
            hi = mid
        else:
            lo = mid
        if hi - lo <= 1e-13 * max(1.0, abs(mid)):
            break
    return beta * 0.5 * (lo + hi)


def pacc_predicted(dM_ins, dM_del, beta, beta_mu):
    """Eq. (21): the mean Metropolis acceptance of insertions,
    <min(1, exp(-beta dM + beta mu))>, and of deletions,
    <min(1, exp(beta dM - beta mu))>, over the sampled work values."""
    a = np.asarray(dM_ins, dtype=np.float64)
    b = np.asarray(dM_del, dtype=np.float64)
    p_ins = float(np.mean(np.exp(np.minimum(0.0, -beta * a[np.isfinite(a)] + beta_mu)))) if len(a) else None
    p_del = float(np.mean(np.exp(np.minimum(0.0, beta * b[np.isfinite(b)] - beta_mu)))) if len(b) else None
    return p_ins, p_del


def alpha2(dM, beta):
    """Non-Gaussianity of a work distribution:
    <(beta dM')^4> / (3 <(beta dM')^2>^2) - 1 with dM' = dM - <dM>
    (0 for a Gaussian, > 0 for fatter tails)."""
    x = np.asarray(dM, dtype=np.float64)
    x = beta * (x[np.isfinite(x)] - np.mean(x[np.isfinite(x)]))
    m2 = np.mean(x * x)
    return float(np.mean(x ** 4) / (3.0 * m2 * m2) - 1.0) if m2 > 0 else None


def overlap_ratio(dM_ins, dM_del, beta_mu, beta):
    """R_ov of Eq. (21): the share of the moves that the Metropolis rule
    accepts for certain, insertions with dM <= mu and deletions with
    dM >= mu (the part of each work distribution past the other's side
    of mu; P_acc is R_ov plus the exponentially weighted rest)."""
    a = np.asarray(dM_ins, dtype=np.float64)
    b = np.asarray(dM_del, dtype=np.float64)
    mu = beta_mu / beta
    r_ins = float(np.mean(a[np.isfinite(a)] <= mu)) if len(a) else None
    r_del = float(np.mean(b[np.isfinite(b)] >= mu)) if len(b) else None
    return r_ins, r_del


def work_summary(dM_ins, dM_del, beta, beta_mu, boot=200, seed=5):
    """Everything the work distributions of one fixed state tell: beta mu
    from BAR (with a 90 % bootstrap interval), the acceptance Eq. (21)
    predicts at the operating beta mu and its certain part R_ov, and the
    mean, variance and alpha_2 of beta dM for each kind of move."""
    a = np.asarray(dM_ins, dtype=np.float64)
    b = np.asarray(dM_del, dtype=np.float64)
    a, b = a[np.isfinite(a)], b[np.isfinite(b)]
    out = {"insertions": int(len(a)), "deletions": int(len(b))}
    for key, x in (("ins", a), ("del", b)):
        out[f"beta_dM_mean_{key}"] = float(beta * np.mean(x)) if len(x) else None
        out[f"beta_dM_var_{key}"] = float(beta * beta * np.var(x)) if len(x) > 1 else None
        out[f"alpha2_{key}"] = alpha2(x, beta) if len(x) > 1 else None
    p_ins, p_del = pacc_predicted(a, b, beta, beta_mu)
    r_ins, r_del = overlap_ratio(a, b, beta_mu, beta)
    out.update(p_acc_ins=p_ins, p_acc_del=p_del, r_ov_ins=r_ins, r_ov_del=r_del)
    if len(a) and len(b):
        est = bar_beta_mu(a, b, beta)
        rng = np.random.default_rng(seed)
        reps = [bar_beta_mu(rng.choice(a, len(a)), rng.choice(b, len(b)), beta) for _ in range(boot)]
        out["beta_mu_bar"] = float(est)
        out["beta_mu_bar_bootstrap90"] = [float(np.percentile(reps, 5)), float(np.percentile(reps, 95))]
    return out
