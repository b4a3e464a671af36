"""Parity bars of the GPU tests (the HIP march against the FP64 oracle).

* Envelopes, relative L2 over the pair (psi+, psi-): FP64 1e-10, FP32 1e-4.
* FP32 R and T: 1e-5 absolute each.
* FP64 R and T: the stated FP64 tolerance bounds the envelopes only.  With
  psi = psi_o + d and |d| <= tol |psi_o| over the pair, a detector power
  changes by at most (2 |psi_o|_D |d| + |d|^2) / P_in <= 2 tol sqrt(X) + tol^2
  for X = R or T, which is the FP64 bar on each.
"""
import math

ENV = {"f64": 1e-10, "f32": 1e-4}
# TOL[prec][0]: the envelope bar (the R and T bars depend on the value: rt_bar)
TOL = {p: (v,) for p, v in ENV.items()}


def env_bar(prec):
    return ENV[prec]


def rt_bar(prec, x_oracle):
    """Bar on |X - X_oracle| for X = R or T."""
    if prec == "f32":
        return 1e-5
    tol = ENV["f64"]
    return 2 * tol * math.sqrt(max(float(x_oracle), 0.0)) + tol * tol


def r_bar(prec, r_oracle):
    return rt_bar(prec, r_oracle)


def t_bar(prec, t_oracle):
    return rt_bar(prec, t_oracle)
