"""Autofocus loss of an image and its cotangent, float64 (test infrastructure).

Reading (the paper names entropy as an autofocus quality measure among others
in Sec. I and defines no loss):
    L(f) = H(f) + ||f - f_clean||^2 / ||f_clean||^2,
    H(f) = -sum_v q_v ln q_v,   q_v = |f_v|^2 / sum_u |f_u|^2.
The cotangent follows the convention g = dL/dRe f + j dL/dIm f:
    g = 2 (dL/d|f|^2) f,  dH/d|f_v|^2 = -(ln q_v + H) / sum_u |f_u|^2.
"""
import numpy as np


def loss(f, f_clean):
    f = np.asarray(f, np.complex128).ravel()
    fc = np.asarray(f_clean, np.complex128).ravel()
    a = np.abs(f) ** 2
    E = a.sum()
    q = a / E
    nz = q > 0
    H = -np.sum(q[nz] * np.log(q[nz]))
    return float(H + np.sum(np.abs(f - fc) ** 2) / np.sum(np.abs(fc) ** 2))


def loss_cotangent(f, f_clean):
    shape = np.shape(f)
    f = np.asarray(f, np.complex128).ravel()
    fc = np.asarray(f_clean, np.complex128).ravel()
    a = np.abs(f) ** 2
    E = a.sum()
    q = a / E
    nz = q > 0
    H = -np.sum(q[nz] * np.log(q[nz]))
    lnq = np.zeros_like(q)
    lnq[nz] = np.log(q[nz])
    dH_da = -(lnq + H) / E
    g = 2.0 * dH_da * f + 2.0 * (f - fc) / np.sum(np.abs(fc) ** 2)
    return g.reshape(shape)
