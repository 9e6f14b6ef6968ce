"""Closed-form solution of a separable box-constrained QP (oracle pin).

Problem (an instance of eq. qp): H = diag(h) with h > 0, A = [I_m1 0] (so
x_i = b_i for i < m1) and bounds l_j <= x_j <= u_j on the remaining coordinates,
written as C = [0 I; 0 -I], d = [l; -u].  The objective separates, so

    x_i = b_i (i < m1),        x_j = clip(-c_j / h_j, l_j, u_j) (j >= m1),
    lam_i = h_i b_i + c_i,
    nu_l,j = h_j x_j + c_j      if x_j = l_j, else 0,
    nu_u,j = -(h_j x_j + c_j)   if x_j = u_j, else 0,

from H x + c - A^T lam - C^T nu = 0 (Sec. 2) coordinate by coordinate.
"""
from __future__ import annotations

import numpy as np


def solve(qp):
    h, l, u = qp.meta["h"], qp.meta["l"], qp.meta["u"]
    m1 = qp.m1
    c, b = qp.c, qp.b
    xf = np.clip(-c[m1:] / h[m1:], l, u)
    x = np.concatenate([b, xf])
    lam = h[:m1] * b + c[:m1]
    g = h[m1:] * xf + c[m1:]
    nu_l = np.where(xf == l, g, 0.0)
    nu_u = np.where(xf == u, -g, 0.0)
    return x, lam, np.concatenate([nu_l, nu_u])
