"""Internal-workload scheduling (Sec. III-C): LPT (Alg. 1) and modified Part_Schedule (Alg. 2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Notation of the paper: tasks T_i with durations tau(T_i); P identical
processors; schedule C with rows c_{p,t}; finish time F_p (12); length
C_max = max_p F_p.  Workload estimate W_i = N_{E,i}^2 and tau = W_i / P_i.

Readings where the listing is terse:
  * ties in "processor with earliest F_p" go to the lowest processor index,
    and the task order is a stable sort by decreasing tau;
  * in Part_Schedule, parallel tasks (P_i > 1) start together at time 0 on
    disjoint processor groups, then sequential tasks are placed by LPT on the
    remaining processors (the condition sum_{P_i>1} P_i <= P of the text);
  * the increment d is 1 below P_cutoff (strict "<", as in the listing), and
    otherwise the distance to the next larger approximate square
    (Q^2 or Q(Q+1)); the budget a is updated exactly as listed.
"""
from __future__ import annotations

import itertools

import numpy as np


def lpt(tau, P):
    """Alg. 1: tasks in decreasing tau, each to the processor with the earliest F_p."""
    order = sorted(range(len(tau)), key=lambda i: (-tau[i], i))
    F = [0.0] * P
    C = [[] for _ in range(P)]
    for i in order:
        p = min(range(P), key=lambda q: (F[q], q))
        C[p].append(i)
        F[p] += tau[i]
    return C, max(F) if P else 0.0


def lpt_bound(P):
    """Worst-case ratio (13) of LPT."""
    return 4.0 / 3.0 - 1.0 / (3.0 * P)


def part_schedule_bound(P):
    """Worst-case ratio (14) of Part_Schedule."""
    return 2.0 / (1.0 - 1.0 / P)


def brute_force_opt(tau, P):
    """Optimal makespan of sequential tasks by enumeration (tiny instances)."""
    best = float('inf')
    n = len(tau)
    for assign in itertools.product(range(P), repeat=n):
        if n and assign[0] != 0:
            continue  # symmetry: first task on processor 0
        F = [0.0] * P
        for i, p in enumerate(assign):
            F[p] += tau[i]
        best = min(best, max(F))
    return best


def is_approx_square(p):
    q = int(np.floor(np.sqrt(p)))
    return q * q == p or q * (q + 1) == p


def next_approx_square(p):
    """Distance from p to the smallest approximate square (Q^2 or Q(Q+1)) larger than p."""
    c = p + 1
    while not is_approx_square(c):
        c += 1
    return c - p


def mixed_schedule(W, Pi, P):
    """Length of the schedule with parallel tasks first (disjoint groups at t = 0), then LPT."""
    tau = [W[i] / Pi[i] for i in range(len(W))]
    par = [i for i in range(len(W)) if Pi[i] > 1]
    used = sum(Pi[i] for i in par)
    if used > P:
        return float('inf'), tau
    F = []
    for i in par:
        F += [tau[i]] * Pi[i]
    F += [0.0] * (P - used)
    seq = sorted([i for i in range(len(W)) if Pi[i] == 1], key=lambda i: (-tau[i], i))
    free = list(range(used, P))
    if seq and not free:
        return float('inf'), tau
    for i in seq:
        p = min(free, key=lambda q: (F[q], q))
        F[p] += tau[i]
    return max(F), tau


def part_schedule(W, P, P_cutoff=20, modified=True):
    """Alg. 2 (modified Part_Schedule); modified=False gives unit increments throughout."""
    n = len(W)
    Pi = [1] * n
    Cmax, tau = mixed_schedule(W, Pi, P)
    a = P
    while a > 0:
        i = max(range(n), key=lambda k: (tau[k], -k))
        h = tau[i]
        d = 1 if (Pi[i] < P_cutoff or not modified) else next_approx_square(Pi[i])
        a = a - d - 1 if Pi[i] == 1 else a - d
        if Cmax != h or a < 0:
            break
        Pi[i] += d
        C2, tau2 = mixed_schedule(W, Pi, P)
        if C2 >= Cmax:
            Pi[i] -= d
            break
        Cmax, tau = C2, tau2
    return Pi, Cmax


def ideal_length(W, P):
    """C_ideal = sum W / P (perfect balance)."""
    return float(np.sum(W)) / P
