"""Metrics shared by the parity tests (test infrastructure)."""
import numpy as np

from paper_1608_05794_amd import synth


def rhs_scale(om, y, P):
    """Per-component scale of the source term: gross production + destruction.

    D_k = (W_k / rho) sum_i |nu_ki| (|q_f,i| + |q_r,i|) for species rows and
    D_T = sum_k |H_k| G_k / (rho cp) for the temperature row, where G_k is the
    gross molar rate of species k.  Near partial equilibrium the net rates
    cancel, so relative error is measured against these gross rates.
    """
    nu = np.abs(om.stoich()).astype(float)
    N, n = y.shape
    D = np.zeros((N, n))
    for r in range(n):
        qf, qr, rho, cp, hRT = om.rates(y[:, r], P[r])
        G = nu @ (np.abs(qf) + np.abs(qr))
        D[1:, r] = om.W * G / rho
        H = synth.R_GAS * y[0, r] * hRT
        D[0, r] = np.sum(np.abs(H) * G) / (rho * cp)
    return D


def jac_scaled_error(J_gpu, J_orc, y):
    """max over entries of |dJ_ij| |y_j| / max_j |J_ij y_j| (row-scaled contribution error).

    J_* are [n, N, N]; y is [N, n].
    """
    ys = np.maximum(np.abs(y.T), 1e-12)[:, None, :]          # [n, 1, N]
    contrib = np.abs(J_orc) * ys
    rows = contrib.max(axis=2, keepdims=True) + 1e-300
    return (np.abs(J_gpu - J_orc) * ys / rows).max()


def weighted_error(y_gpu, y_orc, rtol=1e-8, atol=1e-12):
    """max_i |dy_i| / (|y_i| + atol/rtol): the difference in units of the solver's own error
    weights (atol + rtol |y_i|) divided by rtol.  Components below atol/rtol are controlled in
    absolute terms by the step-size controller, so they are compared in absolute terms here."""
    return (np.abs(y_gpu - y_orc) / (np.abs(y_orc) + atol / rtol)).max(initial=0.0)


def state_rel_error(y_gpu, y_orc, y_floor=1e-12):
    """Relative error of T and of every mass fraction above y_floor."""
    eT = np.abs(y_gpu[0] - y_orc[0]) / np.abs(y_orc[0])
    mask = np.abs(y_orc[1:]) > y_floor
    eY = np.where(mask, np.abs(y_gpu[1:] - y_orc[1:]) / np.where(mask, np.abs(y_orc[1:]), 1.0), 0.0)
    return eT.max(initial=0.0), eY.max(initial=0.0)
