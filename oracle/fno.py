"""FP64 oracle of the Fourier-neural-operator surrogate (forward, loss and
hand-derived backward).  TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Architecture (the surrogate advances the velocity by a fixed number of solver
steps; nothing of it is in the paper):
    v0 = Wl u + bl                                  (lift, 3 -> width)
    for l < L:  s_l = Wc_l v_l + bc_l + K_l(v_l)
                v_{l+1} = gelu(s_l) (l < L-1),  s_l (last layer)
    K_l(v) = c2r( R_l . r2c(v) on the retained modes, 0 elsewhere )
    pre = Wq1 v_L + bq1 ;  y = Wq2 gelu(pre) + bq2  (projection width -> hidden -> 3)
    out = u + y
    loss = mean_b ||out_b - t_b|| / ||t_b||
Retained modes: kx in [0, m), ky and kz in [0, m) U [n - m, n) (half spectrum
along x).  R_l[mode][c_in][c_out] is complex.  gelu is the exact erf form.
r2c carries 1/n^3, c2r is unscaled (the oracle's own transforms).

Adjoints used by backward (weighted inner product on half spectra,
<X, Y>_w = sum_k w(k) Re(conj X . Y), w = 1 on kx = 0 or n/2, else 2):
    c2r^T = n^3 r2c  and  r2c^T = c2r / n^3,
so for k = c2r(R V) with V = r2c(v) and upstream gradient g_k:
    ghat = n^3 r2c(g_k),  g_R = w ghat conj(V),  g_v = c2r(conj(R)^T ghat) / n^3.
"""
from __future__ import annotations

import math

import numpy as np

from . import c2r3, r2c3

_SQRT2 = math.sqrt(2.0)
_ERF = np.vectorize(math.erf)


def gelu(x):
    return 0.5 * x * (1.0 + _ERF(x / _SQRT2))


def gelu_grad(x):
    return 0.5 * (1.0 + _ERF(x / _SQRT2)) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def mode_index(n, m):
    """(kz, ky, kx) indices of the retained modes, in the library's mode order:
    kx fastest, then ky, then kz, each full axis ordered [0, m) then [n-m, n)."""
    ax = np.concatenate([np.arange(m), np.arange(n - m, n)])
    kz, ky, kx = np.meshgrid(ax, ax, np.arange(m), indexing="ij")
    return kz.ravel(), ky.ravel(), kx.ravel()


def mode_weights(n, m):
    _, _, kx = mode_index(n, m)
    return np.where((kx == 0) | (2 * kx == n), 1.0, 2.0)


def param_shapes(width, modes, layers, hidden, n):
    nm = (2 * modes) ** 2 * modes
    shp = [("Wl", (width, 3)), ("bl", (width,))]
    for l in range(layers):
        shp += [(f"Wc{l}", (width, width)), (f"bc{l}", (width,)), (f"R{l}", (nm, width, width, 2))]
    shp += [("Wq1", (hidden, width)), ("bq1", (hidden,)), ("Wq2", (3, hidden)), ("bq2", (3,))]
    return shp


def unflatten(theta, width, modes, layers, hidden, n):
    p, off = {}, 0
    for name, shape in param_shapes(width, modes, layers, hidden, n):
        size = int(np.prod(shape))
        a = theta[off:off + size].reshape(shape)
        p[name] = a[..., 0] + 1j * a[..., 1] if name.startswith("R") else a
        off += size
    assert off == theta.size
    return p


def flatten_grads(g, width, modes, layers, hidden, n):
    out = []
    for name, shape in param_shapes(width, modes, layers, hidden, n):
        a = g[name]
        if name.startswith("R"):
            a = np.stack([a.real, a.imag], axis=-1)
        out.append(np.asarray(a, np.float64).reshape(-1))
    return np.concatenate(out)


def _r2c_b(v):
    """v [B][C][n][n][n] -> [B][C][n][n][n/2+1]"""
    return np.stack([np.stack([r2c3(v[b, c]) for c in range(v.shape[1])]) for b in range(v.shape[0])])


def _c2r_b(h, n):
    return np.stack([np.stack([c2r3(h[b, c], n) for c in range(h.shape[1])]) for b in range(h.shape[0])])


def _chan(W, v):
    """apply a channel matrix W [O][C] to v [B][C][...]"""
    return np.einsum("oc,bc...->bo...", W, v)


def _bias(b, nd):
    return b.reshape((1, -1) + (1,) * nd)


def spectral_conv(v, R, n, m):
    kz, ky, kx = mode_index(n, m)
    V = _r2c_b(v)
    Vm = V[:, :, kz, ky, kx]                       # [B][C][modes]
    Wm = np.einsum("mco,bcm->bom", R, Vm)
    H = np.zeros((v.shape[0], R.shape[2]) + V.shape[2:], complex)
    H[:, :, kz, ky, kx] = Wm
    return _c2r_b(H, n), Vm


def forward(theta, u, cfg, keep=False):
    n, width, modes, layers, hidden = cfg["n"], cfg["width"], cfg["modes"], cfg["layers"], cfg["hidden"]
    p = unflatten(theta, width, modes, layers, hidden, n)
    cache = {"u": u}
    v = _chan(p["Wl"], u) + _bias(p["bl"], 3)
    cache["v0"] = v
    for l in range(layers):
        k, Vm = spectral_conv(v, p[f"R{l}"], n, modes)
        s = _chan(p[f"Wc{l}"], v) + _bias(p[f"bc{l}"], 3) + k
        cache[f"s{l}"], cache[f"V{l}"] = s, Vm
        v = gelu(s) if l < layers - 1 else s
        cache[f"v{l + 1}"] = v
    pre = _chan(p["Wq1"], v) + _bias(p["bq1"], 3)
    y = _chan(p["Wq2"], gelu(pre)) + _bias(p["bq2"], 3)
    cache["pre"] = pre
    out = u + y
    return (out, cache, p) if keep else out


def loss(out, tgt):
    B = out.shape[0]
    e = (out - tgt).reshape(B, -1)
    t = tgt.reshape(B, -1)
    return float(np.mean(np.linalg.norm(e, axis=1) / np.linalg.norm(t, axis=1)))


def loss_and_grad(theta, u, tgt, cfg):
    """Loss and its gradient with respect to the flat parameter vector."""
    n, width, modes, layers, hidden = cfg["n"], cfg["width"], cfg["modes"], cfg["layers"], cfg["hidden"]
    out, c, p = forward(theta, u, cfg, keep=True)
    B = u.shape[0]
    e = out - tgt
    en = np.linalg.norm(e.reshape(B, -1), axis=1)
    tn = np.linalg.norm(tgt.reshape(B, -1), axis=1)
    L = float(np.mean(en / tn))
    dout = e / (B * en * tn).reshape(B, 1, 1, 1, 1)
    g = {}
    red = (0, 2, 3, 4)
    # projection
    h = gelu(c["pre"])
    g["Wq2"] = np.einsum("bozyx,bczyx->oc", dout, h)
    g["bq2"] = dout.sum(axis=red)
    dpre = _chan(p["Wq2"].T, dout) * gelu_grad(c["pre"])
    vL = c[f"v{layers}"]
    g["Wq1"] = np.einsum("bozyx,bczyx->oc", dpre, vL)
    g["bq1"] = dpre.sum(axis=red)
    dv = _chan(p["Wq1"].T, dpre)
    kz, ky, kx = mode_index(n, modes)
    w = mode_weights(n, modes)
    P3 = float(n) ** 3
    for l in reversed(range(layers)):
        s = c[f"s{l}"]
        ds = dv * gelu_grad(s) if l < layers - 1 else dv
        vl = c[f"v{l}"]
        g[f"Wc{l}"] = np.einsum("bozyx,bczyx->oc", ds, vl)
        g[f"bc{l}"] = ds.sum(axis=red)
        # spectral branch adjoint
        Gh = P3 * _r2c_b(ds)[:, :, kz, ky, kx]            # ghat [B][O][modes]
        g[f"R{l}"] = np.einsum("m,bom,bcm->mco", w, Gh, np.conj(c[f"V{l}"]))
        gV = np.einsum("mco,bom->bcm", np.conj(p[f"R{l}"]), Gh)
        H = np.zeros((B, width, n, n, n // 2 + 1), complex)
        H[:, :, kz, ky, kx] = gV
        dv = _chan(p[f"Wc{l}"].T, ds) + _c2r_b(H, n) / P3
    g["Wl"] = np.einsum("bozyx,bczyx->oc", dv, u)
    g["bl"] = dv.sum(axis=red)
    return L, flatten_grads(g, width, modes, layers, hidden, n)
