"""Tap lists of common convolution layers for nj_conv_plan_create_taps (Sec. 3.3).

A tap (out_ch, in_ch, dy, dx, w) adds w * in[in_ch][y+dy][x+dx] to out[out_ch][y][x].
Stride 2 is a unit-stride conv over the four phase images of each input channel
(phase (a, b) = rows a::2, columns b::2, stored as channel (2a + b) C_in + i): the
kernel tap at (u, v) with padding p reads phase ((u-p) mod 2, (v-p) mod 2) at offset
(floor((u-p)/2), floor((v-p)/2)).
"""
import numpy as np


def taps_same(K):
    """K [C_out][C_in][f][f], stride 1, 'same' zero padding"""
    co, ci, f, _ = K.shape
    p = (f - 1) // 2
    return [(o, i, u - p, v - p, float(K[o, i, u, v]))
            for o in range(co) for i in range(ci) for u in range(f) for v in range(f)]


def taps_depthwise(K):
    """K [C][f][f], one kernel per channel, stride 1, 'same' zero padding"""
    c, f, _ = K.shape
    p = (f - 1) // 2
    return [(ch, ch, u - p, v - p, float(K[ch, u, v])) for ch in range(c) for u in range(f) for v in range(f)]


def taps_stride2(K):
    """K [C_out][C_in][f][f], stride 2, padding (f-1)/2, on the phase-image inputs"""
    co, ci, f, _ = K.shape
    p = (f - 1) // 2
    out = []
    for o in range(co):
        for i in range(ci):
            for u in range(f):
                dy, a = divmod(u - p, 2)
                for v in range(f):
                    dx, b = divmod(v - p, 2)
                    out.append((o, (2 * a + b) * ci + i, dy, dx, float(K[o, i, u, v])))
    return out


def phase_images(img):
    """[C][w][w] (w even) -> [4C][w/2][w/2], channel (2a + b) C + i = img[i][a::2, b::2]"""
    return np.concatenate([img[:, a::2, b::2] for a in (0, 1) for b in (0, 1)], axis=0)
