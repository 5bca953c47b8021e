"""Writes tests/golden/sas_check.json: hand-derived values of Check
(Algorithm 5 / 8) and of the Stop-and-Stare parameters (equations "lambda",
"lambda_1", "guard" / "nguard" and the lemma bounding the iterations).

Each Check case is chosen so that the scale factor
    |R'_t| (1 + eps) / (2^(t-1) Cov_{R'_t})
is a perfect square (1/4, 1, 4 or 100): eps_2 is then a rational number and
eps_3 a square root of a rational function of 1/e.  The closed forms are
written out per case below, simplified by hand, and evaluated here with
50-digit decimal arithmetic.  The parameter sets use the exact binomial
coefficient (math.comb) for ln C(S, k).

This script does not import the oracle or the library: it is the pin.
Run:  python tests/golden/make_sas_check.py
"""
import json
import math
import os
from decimal import Decimal as D, getcontext

getcontext().prec = 50
E = D(1).exp()
INV_E = 1 / E
E1 = 1 - INV_E  # 1 - 1/e


def s(x):
    """Decimal -> string with 30 significant digits."""
    return format(+x, ".30g")


def check_cases():
    cases = []

    # A: eps = 1/2, t = 1, |R'| = 8, Cov' = 3, Cov = 3, Lambda_1 = 3.
    #    scale = 8 * (3/2) / (1 * 3) = 4, eps_1 = 0, eps_2 = (1/2) * 2 = 1,
    #    eps_3 = (1/2) * sqrt(4 (1/2 - 1/e) / (7/6)) = sqrt(6 (1/2 - 1/e) / 7),
    #    eps_t = (1/2 - 1/e) + (1 - 1/e) eps_3.  Cov' = Lambda_1: the cut-off
    #    test (Cov' >= Lambda_1) passes on equality.
    e3 = (6 * (D(1) / 2 - INV_E) / 7).sqrt()
    et = (D(1) / 2 - INV_E) + E1 * e3
    cases.append(dict(name="A", eps="1/2", t=1, n_rp=8, cov_rp=3, cov_r=3, lambda1=3,
                      closed_form=dict(scale="4", eps1="0", eps2="1", eps3="sqrt(6(1/2-1/e)/7)",
                                       eps_t="(1/2-1/e) + (1-1/e) sqrt(6(1/2-1/e)/7)"),
                      eps1="0", eps2="1", eps3=s(e3), eps_t=s(et), passed=bool(et <= D(1) / 2)))

    # B: eps = 1/2, t = 3, |R'| = 80, Cov' = 30, Cov = 45, Lambda_1 = 30.
    #    scale = 80 (3/2) / (4 * 30) = 1, eps_1 = 45/30 - 1 = 1/2, eps_2 = 1/2,
    #    eps_3 = (1/2) sqrt(6 (1/2 - 1/e) / 7),
    #    eps_t = (1/2 + 1/2 + 1/4)(1/2 - 1/e) + (1 - 1/e) eps_3.
    e3 = (6 * (D(1) / 2 - INV_E) / 7).sqrt() / 2
    et = D(5) / 4 * (D(1) / 2 - INV_E) + E1 * e3
    cases.append(dict(name="B", eps="1/2", t=3, n_rp=80, cov_rp=30, cov_r=45, lambda1=30,
                      closed_form=dict(scale="1", eps1="1/2", eps2="1/2", eps3="(1/2) sqrt(6(1/2-1/e)/7)",
                                       eps_t="(5/4)(1/2-1/e) + (1-1/e)(1/2) sqrt(6(1/2-1/e)/7)"),
                      eps1="0.5", eps2="0.5", eps3=s(e3), eps_t=s(et), passed=bool(et <= D(1) / 2)))

    # C: case B with Lambda_1 = 31 > Cov' = 30: Check returns False before
    #    forming eps_t.
    cases.append(dict(name="C", eps="1/2", t=3, n_rp=80, cov_rp=30, cov_r=45, lambda1=31,
                      closed_form=dict(note="Cov' = 30 < Lambda_1 = 31"),
                      eps1=None, eps2=None, eps3=None, eps_t=None, passed=False))

    # D: eps = 1/10, t = 2, |R'| = 2000, Cov' = 11, Cov = 10, Lambda_1 = 11.
    #    scale = 2000 (11/10) / (2 * 11) = 100, eps_1 = 10/11 - 1 = -1/11,
    #    eps_2 = (1/10) * 10 = 1,
    #    eps_3 = (1/10) sqrt(100 (9/10 - 1/e) / (31/30)) = sqrt(30 (9/10 - 1/e) / 31),
    #    eps_t = (-1/11 + 1 - 1/11)(9/10 - 1/e) + (1 - 1/e) eps_3
    #          = (9/11)(9/10 - 1/e) + (1 - 1/e) eps_3 > 1/10: fails.
    e3 = (30 * (D(9) / 10 - INV_E) / 31).sqrt()
    et = D(9) / 11 * (D(9) / 10 - INV_E) + E1 * e3
    cases.append(dict(name="D", eps="1/10", t=2, n_rp=2000, cov_rp=11, cov_r=10, lambda1=11,
                      closed_form=dict(scale="100", eps1="-1/11", eps2="1", eps3="sqrt(30(9/10-1/e)/31)",
                                       eps_t="(9/11)(9/10-1/e) + (1-1/e) sqrt(30(9/10-1/e)/31)"),
                      eps1=s(D(-1) / 11), eps2="1", eps3=s(e3), eps_t=s(et), passed=bool(et <= D(1) / 10)))

    # E: eps = 1/10, t = 5, |R'| = 4000, Cov' = 1100, Cov = 1100, Lambda_1 = 1000.
    #    scale = 4000 (11/10) / (16 * 1100) = 1/4, eps_1 = 0, eps_2 = 1/20,
    #    eps_3 = (1/20) sqrt(30 (9/10 - 1/e) / 31),
    #    eps_t = (1/20)(9/10 - 1/e) + (1 - 1/e) eps_3 <= 1/10: passes.
    e3 = (30 * (D(9) / 10 - INV_E) / 31).sqrt() / 20
    et = (D(9) / 10 - INV_E) / 20 + E1 * e3
    cases.append(dict(name="E", eps="1/10", t=5, n_rp=4000, cov_rp=1100, cov_r=1100, lambda1=1000,
                      closed_form=dict(scale="1/4", eps1="0", eps2="1/20", eps3="(1/20) sqrt(30(9/10-1/e)/31)",
                                       eps_t="(1/20)(9/10-1/e) + (1-1/e)(1/20) sqrt(30(9/10-1/e)/31)"),
                      eps1="0", eps2="0.05", eps3=s(e3), eps_t=s(et), passed=bool(et <= D(1) / 10)))
    return cases


def param_set(name, S, k, eps_num, eps_den, delta_num, delta_den, note):
    """Parameters for (S, k, eps, delta) with eps, delta rational.

    c = 2 + 2 eps / 3; with eps = a/b:
      Upsilon(eps, delta/3) = c ln(3/delta) / eps^2
      N_max  = (2 - 1/e)^2 c S (ln(6/delta) + ln C(S,k)) / (k eps^2)
      t_max  = ceil(log2(2 N_max / Upsilon))
             = ceil(log2(2 (2 - 1/e)^2 S (ln(6/delta) + ln C(S,k)) / (k ln(3/delta))))
               (c and eps cancel)
      Lambda   = c ln(3 t_max / delta) / eps^2
      Lambda_1 = 1 + (1 + eps) Lambda
    """
    eps = D(eps_num) / D(eps_den)
    delta = D(delta_num) / D(delta_den)
    c = 2 + 2 * eps / 3
    ln_c = D(math.comb(S, k)).ln()
    two_minus = 2 - INV_E
    n_max = two_minus * two_minus * c * S * ((6 / delta).ln() + ln_c) / (k * eps * eps)
    ratio = 2 * two_minus * two_minus * S * ((6 / delta).ln() + ln_c) / (k * (3 / delta).ln())
    log2_ratio = ratio.ln() / D(2).ln()
    t_max = int(log2_ratio.to_integral_value(rounding="ROUND_CEILING"))
    lam = c * (3 * t_max / delta).ln() / (eps * eps)
    lam1 = 1 + (1 + eps) * lam
    return dict(name=name, note=note, S=S, k=k, eps=f"{eps_num}/{eps_den}", delta=f"{delta_num}/{delta_den}",
                ln_binom=s(ln_c), log2_ratio=s(log2_ratio), upsilon=s(c * (3 / delta).ln() / (eps * eps)),
                n_max=s(n_max), t_max=t_max, lam=s(lam), lam1=s(lam1))


def main():
    out = dict(
        citation=("Check: Algorithm 5 (edges) / Algorithm 8 (nodes) -- eps_1, eps_2, eps_3, eps_t and the "
                  "Lambda_1 cut-off; parameters: equations 'lambda', 'lambda_1', 'guard' (edges, S = m) and "
                  "'nguard' (nodes, S = n); t_max from the lemma bounding the iterations, which uses "
                  "Upsilon(eps, delta/3) = (2 + 2eps/3) ln(3/delta) / eps^2 (the displayed t_max takes "
                  "ln(delta/3) < 0 and is read through the lemma); N_t = ceil(Lambda 2^(t-1))"),
        derivation=("Check cases: scale = |R'_t|(1+eps)/(2^(t-1) Cov_{R'_t}) is made a perfect square so that "
                    "eps_2 = eps sqrt(scale) is rational and eps_3 = eps sqrt(scale (1-1/e-eps)/(1+eps/3)) "
                    "is the square root of a rational function of 1/e; the simplified closed form of each "
                    "quantity is listed with the case.  Parameter sets: ln C(S,k) from the exact integer "
                    "binomial, everything evaluated in 50-digit decimal arithmetic; t_max is the ceiling of "
                    "log2_ratio, in which eps cancels."),
        generator="tests/golden/make_sas_check.py (50-digit decimal arithmetic; imports neither the oracle "
                  "nor the library)",
        check=check_cases(),
        params=[
            param_set("er1k_nodes", 1000, 10, 1, 2, 1, 1000,
                      "nSIA on the 1000-node, 8000-edge G(n,m) workload: S = n, k = 10, eps = 1/2, delta = 1/n"),
            param_set("er1k_edges", 8000, 10, 1, 10, 1, 1000,
                      "eSIA on the same workload: S = m, k = 10, eps = 1/10, delta = 1/n"),
            param_set("rmat24_edges", 263_430_593, 1000, 1, 10, 1, 16_777_216,
                      "eSIA on R-MAT scale 24 after cleanup: S = m = 263430593, k = 1000, eps = 1/10, "
                      "delta = 1/n = 2^-24"),
        ],
    )
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sas_check.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
