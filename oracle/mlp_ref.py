"""FP64 reference of the small network that proposes the initial star pressure
of the exact Riemann solve.  TEST INFRASTRUCTURE ONLY (see oracle/__init__).

The network and its inputs (the paper is silent here; these are the readings
the design notes list):
  inputs  the face states as deviations from their mean, normalised by it:
          x = (rho_L/rho_m - 1, (u_L - u_m)/a_m, p_L/p_m - 1,
               rho_R/rho_m - 1, (u_R - u_m)/a_m, p_R/p_m - 1)
          with rho_m, u_m, p_m the means of the two sides,
          a_m = sqrt(gamma p_m / rho_m), u the face-normal velocities
          (x_3 = -x_0, x_4 = -x_1, x_5 = -x_2).  The Euler equations are
          invariant under rho -> s rho, u -> c u, p -> s c^2 p and under a
          shift of u, which leave x and ln(p*/p_m) unchanged, so the target
          is a function of x alone.  Deviations rather than ratios: weak
          waves differ from the mean by little, and BF16 keeps 8 bits of a
          small deviation but only 8 bits of a ratio near 1;
  network h1 = relu(W1 x + b1) (32), h2 = relu(W2 h1 + b2) (32),
          y = w3 . h2 + b3, a correction of the two-rarefaction value p_TR
          (Toro, ch. 4): the guess is p0 = p_TR exp(y);
  target  y* = ln(p*/p_TR), also invariant under the scaling above;
  loss    mean squared error of y over a batch.
Parameter vector (1313 values): W1 [32][6] row-major, b1 [32], W2 [32][32]
row-major, b2 [32], w3 [32], b3.

The BF16-emulating forward rounds inputs (after an FP32 rounding of the
features), weights, biases and the two hidden activations to BF16 with
round-to-nearest-even, and accumulates in FP64; the BF16-emulating backward
also rounds the back-propagated gradients dz2 and dz1 to BF16 (the operands
of the training products).
"""
import numpy as np

N_IN, N_H = 6, 32
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
         ("w3", (N_H,)), ("b3", ())]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)  # 1313


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,)
    out, k = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[k:k + n].reshape(shape) if shape else theta[k]
        k += n
    return out


def pack(p):
    return np.concatenate([np.ravel(np.asarray(p[name], dtype=np.float64)) for name, _ in SIZES])


def bf16(x):
    """Round to bfloat16 (round to nearest, ties to even) via FP32, as float64."""
    x32 = np.asarray(x, dtype=np.float32)
    bits = x32.view(np.uint32).astype(np.uint64)
    rounded = ((bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return rounded.view(np.float32).astype(np.float64)


def features(wl, wr, gamma=1.4):
    """wl, wr: [n][3] (rho, u_n, p) -> x [n][6] and the normalisers (rho_m, p_m, a_m)."""
    wl = np.atleast_2d(np.asarray(wl, dtype=np.float64))
    wr = np.atleast_2d(np.asarray(wr, dtype=np.float64))
    rm = 0.5 * (wl[:, 0] + wr[:, 0])
    um = 0.5 * (wl[:, 1] + wr[:, 1])
    pm = 0.5 * (wl[:, 2] + wr[:, 2])
    am = np.sqrt(gamma * pm / rm)
    x = np.stack([wl[:, 0] / rm - 1.0, (wl[:, 1] - um) / am, wl[:, 2] / pm - 1.0,
                  wr[:, 0] / rm - 1.0, (wr[:, 1] - um) / am, wr[:, 2] / pm - 1.0], axis=1)
    return x, rm, pm, am


def two_rarefaction(wl, wr, gamma=1.4):
    """p_TR = [(a_L + a_R - (g-1)/2 (u_R - u_L)) / (a_L p_L^-z + a_R p_R^-z)]^(1/z),
    z = (g-1)/(2g): the star pressure if both waves are rarefactions."""
    wl = np.atleast_2d(np.asarray(wl, dtype=np.float64))
    wr = np.atleast_2d(np.asarray(wr, dtype=np.float64))
    z = (gamma - 1.0) / (2.0 * gamma)
    al = np.sqrt(gamma * wl[:, 2] / wl[:, 0])
    ar = np.sqrt(gamma * wr[:, 2] / wr[:, 0])
    num = al + ar - 0.5 * (gamma - 1.0) * (wr[:, 1] - wl[:, 1])
    den = al * wl[:, 2] ** (-z) + ar * wr[:, 2] ** (-z)
    return (num / den) ** (1.0 / z)


def target(p_star, p_tr):
    """ln(p*/p_TR)."""
    return np.log(np.asarray(p_star, dtype=np.float64) / p_tr)


def forward(theta, x, emulate_bf16=False):
    """Returns y [n] and the activations needed by backward()."""
    p = unpack(theta)
    x = np.asarray(x, dtype=np.float64)
    if emulate_bf16:
        x = bf16(x)
        p = {k: bf16(v) for k, v in p.items()}
    z1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    if emulate_bf16:
        h1 = bf16(h1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    if emulate_bf16:
        h2 = bf16(h2)
    y = h2 @ p["w3"] + p["b3"]
    return y, dict(x=x, z1=z1, h1=h1, z2=z2, h2=h2, p=p)


def loss(theta, x, t, emulate_bf16=False):
    y, _ = forward(theta, x, emulate_bf16)
    return float(np.mean((y - t) ** 2))


def backward(theta, x, t, emulate_bf16=False):
    """Gradient of the mean squared error with respect to the parameter
    vector (chain rule through the ReLU network, FP64).

    With emulate_bf16 the forward pass is the BF16 one above, and the two
    back-propagated pre-activation gradients dz2 and dz1 are rounded to BF16
    once formed (after the ReLU mask), because they are operands of the
    BF16-in / FP32-accumulate products of training (dW2 = dz2^T h1,
    dh1 = dz2 W2, dW1 = dz1^T x); the bias gradients are sums of those
    rounded values.  dy and the last layer's products stay unrounded."""
    y, a = forward(theta, x, emulate_bf16)
    p = a["p"]
    n = len(y)
    dy = 2.0 * (y - t) / n
    g = {}
    g["w3"] = a["h2"].T @ dy
    g["b3"] = dy.sum()
    dz2 = np.outer(dy, p["w3"]) * (a["z2"] > 0)
    if emulate_bf16:
        dz2 = bf16(dz2)
    g["W2"] = dz2.T @ a["h1"]
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"]) * (a["z1"] > 0)
    if emulate_bf16:
        dz1 = bf16(dz1)
    g["W1"] = dz1.T @ a["x"]
    g["b1"] = dz1.sum(0)
    return pack(g)


def he_uniform(seed):
    """He-uniform initial parameters (biases 0) from a seeded generator."""
    rng = np.random.default_rng(seed)
    p = {}
    lim1 = np.sqrt(6.0 / N_IN)
    lim2 = np.sqrt(6.0 / N_H)
    p["W1"] = rng.uniform(-lim1, lim1, (N_H, N_IN))
    p["b1"] = np.zeros(N_H)
    p["W2"] = rng.uniform(-lim2, lim2, (N_H, N_H))
    p["b2"] = np.zeros(N_H)
    p["w3"] = rng.uniform(-lim2, lim2, N_H)
    p["b3"] = 0.0
    return pack(p)
