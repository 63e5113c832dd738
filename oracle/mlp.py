"""Temperature-guess MLP: forward, backward and Adam (oracle).

The method's iterative thermochemistry (Introduction; Appendix,
Thermodynamics) needs an initial temperature for every per-node T(e) solve.
The learned guess is a 6 -> 64 -> 64 -> 64 -> 1 network with tanh hidden
layers:

  features  x = ((log10 max(rho_s, 1e-30))_{s=1..5}, e) standardised with
            stored means/standard deviations, e = rho e / rho the specific
            internal energy;
  output    y = standardised temperature, T_guess = y * T_std + T_mean.

Reading (the workload fixes BF16 matrix operands with FP32 accumulation but
not the exact rounding points): the oracle evaluates in FP64 and rounds to
BF16 (round to nearest even) exactly where the GPU kernels feed a matrix
unit: the standardised features, the weights W1..W3 and the hidden
activations h1, h2 entering the next layer; in the backward pass the
back-propagated dz3, dz2, dz1 wherever they enter a matrix product
(W^T dz and dz h^T).  Biases, tanh, the output layer
(W4 . h3 with h3 unrounded) and the loss are FP32 on the GPU and FP64 here.
Loss: mean squared error of y against the standardised target.  Adam with
beta1 = 0.9, beta2 = 0.999, eps = 1e-8 on FP32 master weights.

Parameter vector (8833 entries): W1[64][6], b1[64], W2[64][64], b2[64],
W3[64][64], b3[64], W4[64], b4; then 14 normalisation entries:
mean[6], std[6], T_mean, T_std.
"""
import numpy as np

H = 64
NIN = 6
SIZES = [("W1", (H, NIN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)), ("b3", (H,)),
         ("W4", (H,)), ("b4", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)
NNORM = 14


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(x, np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    r = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(theta):
    out = {}
    o = 0
    for name, shp in SIZES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], np.float64).reshape(shp)
        o += n
    norm = np.asarray(theta[NPARAM:NPARAM + NNORM], np.float64)
    out["mean"], out["std"], out["Tm"], out["Ts"] = norm[:6], norm[6:12], norm[12], norm[13]
    return out


def pack(p):
    return np.concatenate([np.ravel(p[name]) for name, _ in SIZES])


def raw_features(rs, rhoe):
    """(count, 6): log10 of each species density (floored) and specific e."""
    rho = rs.sum(0)
    f = [np.log10(np.maximum(rs[s], 1e-30)) for s in range(5)]
    f.append(rhoe / rho)
    return np.stack(f, 1)


def standardise(raw, p):
    return np.asarray((raw - p["mean"]) / p["std"], np.float32).astype(np.float64)


def init_params(seed=41):
    """Glorot-uniform weights, zero biases (FP32 master copy)."""
    rng = np.random.default_rng(seed)
    theta = []
    for name, shp in SIZES:
        if name.startswith("W"):
            fan_in = shp[-1] if len(shp) == 2 else H
            fan_out = shp[0] if len(shp) == 2 else 1
            lim = np.sqrt(6.0 / (fan_in + fan_out))
            theta.append(rng.uniform(-lim, lim, int(np.prod(shp))))
        else:
            theta.append(np.zeros(int(np.prod(shp))))
    return np.concatenate(theta).astype(np.float32)


def forward(p, x):
    """x: (count, 6) standardised features.  Returns y and the cache."""
    xb = bf16(x)
    z1 = xb @ bf16(p["W1"]).T + p["b1"]
    h1 = np.tanh(z1)
    z2 = bf16(h1) @ bf16(p["W2"]).T + p["b2"]
    h2 = np.tanh(z2)
    z3 = bf16(h2) @ bf16(p["W3"]).T + p["b3"]
    h3 = np.tanh(z3)
    y = h3 @ p["W4"] + p["b4"][0]
    return y, dict(xb=xb, h1=h1, h2=h2, h3=h3)


def loss_and_grad(p, x, t):
    """Mean squared error and its gradient with respect to every parameter."""
    y, c = forward(p, x)
    n = x.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / n
    g = {}
    g["W4"] = c["h3"].T @ dy
    g["b4"] = np.array([dy.sum()])
    dz3 = np.outer(dy, p["W4"]) * (1.0 - c["h3"] ** 2)
    g["W3"] = bf16(dz3).T @ bf16(c["h2"])
    g["b3"] = dz3.sum(0)
    dz2 = (bf16(dz3) @ bf16(p["W3"])) * (1.0 - c["h2"] ** 2)
    g["W2"] = bf16(dz2).T @ bf16(c["h1"])
    g["b2"] = dz2.sum(0)
    dz1 = (bf16(dz2) @ bf16(p["W2"])) * (1.0 - c["h1"] ** 2)
    g["W1"] = bf16(dz1).T @ c["xb"]
    g["b1"] = dz1.sum(0)
    return loss, g


def loss_and_grad_exact(p, x, t):
    """The same network without any BF16 rounding (for finite differences)."""
    z1 = x @ p["W1"].T + p["b1"]
    h1 = np.tanh(z1)
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    h3 = np.tanh(h2 @ p["W3"].T + p["b3"])
    y = h3 @ p["W4"] + p["b4"][0]
    n = x.shape[0]
    r = y - t
    dy = 2.0 * r / n
    g = {"W4": h3.T @ dy, "b4": np.array([dy.sum()])}
    dz3 = np.outer(dy, p["W4"]) * (1.0 - h3 ** 2)
    g["W3"], g["b3"] = dz3.T @ h2, dz3.sum(0)
    dz2 = (dz3 @ p["W3"]) * (1.0 - h2 ** 2)
    g["W2"], g["b2"] = dz2.T @ h1, dz2.sum(0)
    dz1 = (dz2 @ p["W2"]) * (1.0 - h1 ** 2)
    g["W1"], g["b1"] = dz1.T @ x, dz1.sum(0)
    return float(np.mean(r * r)), g


def adam_step(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
