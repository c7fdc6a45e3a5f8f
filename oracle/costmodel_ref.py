"""Oracle of the subdivision cost model (test infrastructure only).

Written term by term from Sec. 4 of the paper, in plain Python floats
(binary64), one level at a time, from the general expressions before they are
specialised: the work of level i is K_i = E[|G_i|] U_i with
E[|G_i|] = G R^i prod_{j<i} P_j and U_i = P_i (Q_i + S) + (1 - P_i)(Q_i + T_i)
(Sec. 4.2); the last level costs L = (n^2 / (G R^{tau-1})) A G R^{tau-1}
prod_{j<=tau-2} P_j; the Mandelbrot terms are Q_i = 4 n A / (g r^i),
T_i = n^2 / (G R^i), S = lambda A (Sec. 4.2.1); the times apply the SBR and
MBR schemes of Sec. 4.3.1 and 4.3.2 with q multiprocessors of c cores.
"""
import math


def tau(n, g, r, B):
    """Depth tau = log_r(n / (g B)) of Sec. 4.2.1 (assumption iii), rounded
    to the nearest integer and at least 1."""
    return max(1, int(round(math.log(n / (g * B)) / math.log(r))))


def work_exhaustive(n, A):
    """W_E = n^2 A (Sec. 4.1)."""
    return float(n) * n * A


def _probs(P, levels):
    return list(P) if isinstance(P, (list, tuple)) else [P] * levels


def work_subdivision(n, g, r, B, A, P, lam):
    """W_S = sum_{i=0}^{tau-2} K_i + L (Sec. 4.2), with per-level P_i
    (a list) or one P for every level (Sec. 4.2.1, assumption i)."""
    t = tau(n, g, r, B)
    G, R = g * g, r * r
    Ps = _probs(P, t)
    total = 0.0
    for i in range(t - 1):
        expected_regions = G * R ** i
        for j in range(i):
            expected_regions *= Ps[j]
        Q = 4.0 * n * A / (g * r ** i)
        T = float(n) * n / (G * R ** i)
        S = lam * A
        U = Ps[i] * (Q + S) + (1.0 - Ps[i]) * (Q + T)
        total += expected_regions * U
    last_regions = G * R ** (t - 1)
    for j in range(t - 1):
        last_regions *= Ps[j]
    total += (float(n) * n / (G * R ** (t - 1))) * A * last_regions
    return total


def reduction_factor(n, g, r, B, A, P, lam):
    """Omega = W_E / W_SSD^M (Sec. 4.2.2)."""
    return work_exhaustive(n, A) / work_subdivision(n, g, r, B, A, P, lam)


def time_exhaustive(n, A, q, c):
    """T_Ex = ceil(n^2 / (q c)) A (Sec. 4.3)."""
    return math.ceil(float(n) * n / (q * c)) * A


def time_sbr(n, g, r, B, A, P, lam, q, c):
    """T_SBR (Sec. 4.3.1): every region on one block of c cores, the regions
    of a level spread over q multiprocessors."""
    t = tau(n, g, r, B)
    G, R = g * g, r * r
    total = 0.0
    for i in range(t - 1):
        per_region = (math.ceil(4.0 * n / (g * r ** i * c)) * A + P * lam * A
                      + (1.0 - P) * math.ceil(float(n) * n / (G * R ** i * c)))
        total += per_region * math.ceil(G * R ** i / q) * P ** i
    last = t - 1
    total += (A * math.ceil(float(n) * n / (G * R ** last * c))
              * math.ceil(G * R ** last / q) * P ** last)
    return total


def time_mbr(n, g, r, B, A, P, lam, q, c):
    """T_MBR (Sec. 4.3.2): queries and splits one block per region, fills and
    the last level spread over all q c cores."""
    t = tau(n, g, r, B)
    G, R = g * g, r * r
    S = lam * A
    total = 0.0
    for i in range(t - 1):
        total += math.ceil(4.0 * n / (g * r ** i * c)) * math.ceil(G * R ** i / q) * A * P ** i
        total += math.ceil(G * R ** i / q) * S * P ** (i + 1)
        total += math.ceil(float(n) * n * P ** i * (1.0 - P) / (q * c))
    total += A * math.ceil(float(n) * n / (q * c)) * P ** (t - 1)
    return total


def time_sbr_levels(n, g, r, B, A, P, lam, q, c, sigma=0.0, levels=None):
    """T_SBR of Sec. 4.3.1 in its general form: a split probability P_i per
    level (a list; level i's expected region count is G R^i prod_{j<i} P_j,
    Sec. 4.2, without assumption i) and a cost sigma that every region adds
    on its block beyond the paper's terms (taking the region from the queue
    and publishing its outcome), in the same units as the other terms, over
    tau levels as printed or the given number of levels. With one P for every
    level, sigma = 0 and tau as printed this is time_sbr."""
    t = tau(n, g, r, B) if levels is None else levels
    G, R = g * g, r * r
    Ps = _probs(P, t)
    total = 0.0
    reach = 1.0  # prod_{j<i} P_j
    for i in range(t - 1):
        per_region = (math.ceil(4.0 * n / (g * r ** i * c)) * A + Ps[i] * lam * A
                      + (1.0 - Ps[i]) * math.ceil(float(n) * n / (G * R ** i * c)) + sigma)
        total += per_region * math.ceil(G * R ** i / q) * reach
        reach *= Ps[i]
    last = t - 1
    total += ((A * math.ceil(float(n) * n / (G * R ** last * c)) + sigma)
              * math.ceil(G * R ** last / q) * reach)
    return total
