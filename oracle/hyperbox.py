"""Closed-form support function of a hyper-rectangle -- TEST INFRASTRUCTURE.

Paper Sec. 5.6, Eq. (7): for B = [a_1, b_1] x ... x [a_n, b_n] and a direction
l, max_{x in B} l.x = sum_i l_i h_i with h_i = a_i when l_i < 0 and h_i = b_i
otherwise (for l_i = 0 either bound gives the same product; the "otherwise"
branch is taken).
"""
import numpy as np


def hyperbox_max(lo, hi, l):
    """lo, hi, l: arrays [..., n] (float64).  Returns (value [...], argmax [..., n])."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    l = np.asarray(l, np.float64)
    h = np.where(l < 0, lo, hi)
    return np.sum(l * h, axis=-1), h
