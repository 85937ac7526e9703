"""Learned coarse propagator: a small message-passing network on the coarsest
mesh that corrects the implicit-Euler coarse step (test infrastructure only).

The MGRIT coarse propagator may be any map (Sec. 2.1: a re-discretisation is
one choice among several); with FAS the fixed point stays the fine-grid
solution whatever it is, so a better coarse map only changes the iteration
count.  This module is the plain FP64 definition of the network the library
trains and evaluates, written so that every quantity can be checked by hand.

Propagator over one coarse step from T_k = k dT to T_{k+1}:

    Psi(u) = p + s_out * delta,   p = Phi_IE(u)   (the implicit-Euler step)

Node features (interior nodes of the coarse mesh, F = m + 7 of them):
    u_i / s_u,  p_i / s_u,
    f_i(T_k + j dT/m) / s_f              for j = 0..m  (m + 1 source samples),
    conductor, iron, coil flags,  (r_i - r_in) / (r_out - r_in)
where f_i(t) is the node's entry of the forcing vector at time t (the source
with the sample's amplitude factor and phase shift, start-up ramp included).

Network (width H = 64, L = 3 message-passing layers, tanh):
    h_0 = tanh(x W_in + b_in)
    a_l = A h_{l-1},  (A h)_i = mean of h_j over the mesh neighbours j of i
    h_l = h_{l-1} + tanh(h_{l-1} Ws_l + a_l Wn_l + b_l)
    delta = h_L w_out + b_out
Weights are used rounded to bfloat16 (round to nearest even); the master copy
and the gradients are FP32 on the GPU (FP64 here).

Loss of a batch of S samples: mean over samples and nodes of ((Psi - y)/s_out)^2.
Optimiser: Adam (Kingma and Ba, 2015) with bias correction.

Parameter vector (the order of the library's weight blob):
    [s_u, s_f, s_out, 0]  (scales, not trained)
    W_in [F][H], b_in [H],
    per layer: Ws [H][H], Wn [H][H], b [H],
    w_out [H], b_out [1]
"""

import numpy as np

from . import pwm

H = 64
LAYERS = 3
N_SCALES = 4


def n_features(m):
    return m + 7


def param_shapes(m):
    F = n_features(m)
    shapes = [("scales", (N_SCALES,)), ("W_in", (F, H)), ("b_in", (H,))]
    for l in range(LAYERS):
        shapes += [(f"Ws{l}", (H, H)), (f"Wn{l}", (H, H)), (f"b{l}", (H,))]
    shapes += [("w_out", (H,)), ("b_out", (1,))]
    return shapes


def n_params(m):
    return int(sum(np.prod(s) for _, s in param_shapes(m)))


def unpack(vec, m):
    out, o = {}, 0
    for name, shape in param_shapes(m):
        k = int(np.prod(shape))
        out[name] = np.asarray(vec[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def pack(params, m):
    return np.concatenate([np.asarray(params[name], dtype=np.float64).ravel()
                           for name, _ in param_shapes(m)])


def bf16_round(a):
    """Round FP32 values to bfloat16 (nearest, ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    r = ((bits + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def rounded(params):
    """Weights as the network uses them: every trained entry rounded to bf16."""
    return {k: (v if k == "scales" else bf16_round(v)) for k, v in params.items()}


# --- graph and static node data ---------------------------------------------

def graph(fe):
    """Interior-node adjacency of the P1 mesh: CSR (ptr, idx) without self
    loops, in the interior numbering of MachineFE."""
    mesh = fe.mesh
    full_to_int = -np.ones(mesh.n_nodes, dtype=np.int64)
    full_to_int[fe.free] = np.arange(fe.n)
    nb = [set() for _ in range(fe.n)]
    for t in mesh.tri:
        ids = full_to_int[t]
        for a in range(3):
            for b in range(3):
                if a != b and ids[a] >= 0 and ids[b] >= 0:
                    nb[ids[a]].add(int(ids[b]))
    ptr = np.zeros(fe.n + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(s) for s in nb])
    idx = np.concatenate([np.array(sorted(s), dtype=np.int64) for s in nb])
    return ptr, idx


def aggregate(ptr, idx, h):
    """(A h)_i = mean over neighbours; h [..., n, H]."""
    out = np.zeros_like(h)
    for i in range(len(ptr) - 1):
        nbrs = idx[ptr[i]:ptr[i + 1]]
        out[..., i, :] = h[..., nbrs, :].mean(axis=-2)
    return out


def aggregate_t(ptr, idx, g):
    """A^T g: (A^T g)_j = sum over i with j in N(i) of g_i / deg_i."""
    out = np.zeros_like(g)
    for i in range(len(ptr) - 1):
        nbrs = idx[ptr[i]:ptr[i + 1]]
        out[..., nbrs, :] += g[..., i:i + 1, :] / len(nbrs)
    return out


def node_flags(fe):
    """[n, 4]: conductor, iron, coil flags and the normalised radius."""
    mesh = fe.mesh
    cond = np.asarray(abs(fe.M).sum(axis=1)).ravel() > 0
    iron_full = np.zeros(mesh.n_nodes, dtype=bool)
    for c in np.nonzero(fe.iron_cell)[0]:
        iron_full[mesh.tri[c]] = True
    coil = np.any(fe.F != 0, axis=0)
    r = np.hypot(mesh.xy[fe.free, 0], mesh.xy[fe.free, 1])
    rin = np.hypot(*mesh.xy[0])              # node (0, 0) lies on the inner radius
    rout = np.hypot(*mesh.xy[-1])            # the last node on the outer radius
    rn = (r - rin) / (rout - rin)
    return np.stack([cond, iron_full[fe.free], coil, rn], axis=1).astype(np.float64)


def forcing(fe, src, t, amp=1.0, dphi=0.0):
    """Forcing vectors [len(t), n] of the source with amplitude factor amp and
    phase shift dphi (added to every phase)."""
    from dataclasses import replace
    s = replace(src, amplitude=src.amplitude * amp, phase_offset=src.phase_offset + dphi)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    b = pwm.phase_signals(t, s)                                    # [3, len(t)]
    scale = s.J0 * s.amplitude * pwm.ramp(t, s)
    return scale[:, None] * (b.T @ fe.F)


def features(u, p, k, dT, m, fe, src, flags, scales, amp=None, dphi=None):
    """x [S, n, F] for states u [S, n], IE predictions p [S, n], coarse step
    indices k [S] (input time T_k = k dT)."""
    u = np.atleast_2d(u)
    p = np.atleast_2d(p)
    S, n = u.shape
    amp = np.ones(S) if amp is None else np.asarray(amp, dtype=np.float64)
    dphi = np.zeros(S) if dphi is None else np.asarray(dphi, dtype=np.float64)
    s_u, s_f = scales[0], scales[1]
    x = np.zeros((S, n, n_features(m)))
    x[:, :, 0] = u / s_u
    x[:, :, 1] = p / s_u
    for s in range(S):
        t = k[s] * dT + np.arange(m + 1) * (dT / m)
        x[s, :, 2:m + 3] = forcing(fe, src, t, amp[s], dphi[s]).T / s_f
    x[:, :, m + 3:] = flags[None]
    return x


# --- network ----------------------------------------------------------------

def forward(params, x, p, ptr, idx):
    """Psi [S, n] and the cache for backward.  params are used as given
    (call rounded() first for the bf16 network)."""
    s_out = params["scales"][2]
    h = np.tanh(x @ params["W_in"] + params["b_in"])
    cache = {"x": x, "hs": [h], "as": [], "ts": []}
    for l in range(LAYERS):
        a = aggregate(ptr, idx, h)
        t = np.tanh(h @ params[f"Ws{l}"] + a @ params[f"Wn{l}"] + params[f"b{l}"])
        h = h + t
        cache["as"].append(a)
        cache["ts"].append(t)
        cache["hs"].append(h)
    delta = h @ params["w_out"] + params["b_out"][0]
    return p + s_out * delta, cache


def loss(psi, y, s_out):
    """Mean squared scaled error and its gradient with respect to psi."""
    d = (psi - y) / s_out
    N = d.size
    return float(np.sum(d * d) / N), 2.0 * d / (s_out * N)


def backward(params, cache, dpsi, ptr, idx):
    """Gradients of the loss with respect to every trained parameter (the
    scales get zero)."""
    s_out = params["scales"][2]
    g = {k: np.zeros_like(v) for k, v in params.items()}
    ddelta = s_out * dpsi                                      # [S, n]
    hL = cache["hs"][-1]
    g["w_out"] = np.einsum("snh,sn->h", hL, ddelta)
    g["b_out"] = np.array([ddelta.sum()])
    gh = ddelta[..., None] * params["w_out"]                   # [S, n, H]
    for l in reversed(range(LAYERS)):
        t = cache["ts"][l]
        hp = cache["hs"][l]
        a = cache["as"][l]
        dz = gh * (1.0 - t * t)
        g[f"Ws{l}"] = np.einsum("snh,snk->hk", hp, dz)
        g[f"Wn{l}"] = np.einsum("snh,snk->hk", a, dz)
        g[f"b{l}"] = dz.sum(axis=(0, 1))
        gh = gh + dz @ params[f"Ws{l}"].T + aggregate_t(ptr, idx, dz @ params[f"Wn{l}"].T)
    h0 = cache["hs"][0]
    dz0 = gh * (1.0 - h0 * h0)
    g["W_in"] = np.einsum("snf,snh->fh", cache["x"], dz0)
    g["b_in"] = dz0.sum(axis=(0, 1))
    return g


def adam_step(master, grads, state, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of the master weights (step counts from 1); the scales
    are not trained."""
    out = {}
    for k, w in master.items():
        if k == "scales":
            out[k] = w
            continue
        m_ = state.setdefault(("m", k), np.zeros_like(w))
        v_ = state.setdefault(("v", k), np.zeros_like(w))
        m_ = beta1 * m_ + (1 - beta1) * grads[k]
        v_ = beta2 * v_ + (1 - beta2) * grads[k] ** 2
        state[("m", k)], state[("v", k)] = m_, v_
        mh = m_ / (1 - beta1 ** step)
        vh = v_ / (1 - beta2 ** step)
        out[k] = w - lr * mh / (np.sqrt(vh) + eps)
    return out


def init_params(m, seed, scales):
    """Glorot-uniform hidden weights, zero biases and a zero output layer
    (so that the untrained propagator is exactly the implicit-Euler step)."""
    rng = np.random.default_rng(seed)
    out = {}
    for name, shape in param_shapes(m):
        if name == "scales":
            out[name] = np.asarray(scales, dtype=np.float64)
        elif len(shape) == 2 and name != "w_out":
            lim = np.sqrt(6.0 / (shape[0] + shape[1]))
            out[name] = rng.uniform(-lim, lim, size=shape)
        else:
            out[name] = np.zeros(shape)
    return out
