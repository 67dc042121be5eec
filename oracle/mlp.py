"""Oracle of the learned birth proposal -- TEST INFRASTRUCTURE ONLY.

Plain FP64 numpy: the network that maps one measurement z = (range, bearing)
to a 4-component diagonal Gaussian mixture over the state [x, vx, y, vy], its
training loss (negative log-likelihood of simulated (z, x) pairs) with the
gradient written out by hand, one Adam step, and the mixture table the births
of Eq 6 draw from.  Used by the tests to check the GPU network and to pin
itself (finite differences, closed forms).  Shares no code with the GPU
library.

Definition (every width is a parameter so that the pins can use small nets):
  features    f(z) = ((s_x + r cos th - c_x) / h_x, (s_y + r sin th - c_y) / h_y)
              with c the centre and h the half-widths of the surveillance region
  network     a1 = W1 f + b1, h1 = relu(a1); a2 = W2 h1 + b2, h2 = relu(a2);
              a3 = W3 h2 + b3, h3 = relu(a3); o = W4 h3 + b4  (36 outputs)
  component c uses o[9c .. 9c+8]:
              logit l_c = o[9c]
              mean  m_c = (f_x + o[9c+1], o[9c+2], f_y + o[9c+3], o[9c+4])
              log-std s_c = clip(o[9c+5 .. 9c+8], -12, 6)
  all in the normalised state xi = ((x - c_x)/h_x, vx/sv, (y - c_y)/h_y, vy/sv);
  the density in state units divides by h_x sv h_y sv.
  loss        mean over pairs of -log sum_c softmax(l)_c prod_d N(xi_d; m_cd, exp(s_cd)^2)
Parameters are one flat vector in the order W1 (out-major, [H][2]), b1, W2
([H][H], row = output unit), b2, W3, b3, W4 ([36][H]), b4.
"""
import numpy as np

NCOMP = 4
NOUT = 9 * NCOMP
LOGSTD_MIN, LOGSTD_MAX = -12.0, 6.0
LOG_2PI = np.log(2.0 * np.pi)


def shapes(hidden=128):
    H = hidden
    return [("W1", (H, 2)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
            ("W3", (H, H)), ("b3", (H,)), ("W4", (NOUT, H)), ("b4", (NOUT,))]


def n_params(hidden=128):
    return int(sum(np.prod(s) for _, s in shapes(hidden)))


def unflatten(theta, hidden=128):
    out, o = {}, 0
    for name, s in shapes(hidden):
        k = int(np.prod(s))
        out[name] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(s)
        o += k
    return out


def flatten(d, hidden=128):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in shapes(hidden)])


def scales(p):
    """(offset O, scale S) of the normalised state xi = (x - O) / S."""
    reg = p["region"]
    cx, cy = 0.5 * (reg[0] + reg[1]), 0.5 * (reg[2] + reg[3])
    hx, hy = 0.5 * (reg[1] - reg[0]), 0.5 * (reg[3] - reg[2])
    sv = float(p["birth_sigma_v"])
    return np.array([cx, 0.0, cy, 0.0]), np.array([hx, sv, hy, sv])


def features(p, Z):
    """Network input of each measurement (rows of Z = (range, bearing))."""
    Z = np.asarray(Z, dtype=np.float64).reshape(-1, 2)
    O, S = scales(p)
    px = p["sensor_x"] + Z[:, 0] * np.cos(Z[:, 1])
    py = p["sensor_y"] + Z[:, 0] * np.sin(Z[:, 1])
    return np.stack([(px - O[0]) / S[0], (py - O[2]) / S[2]], axis=1)


def forward(theta, F, hidden=128):
    """Outputs o [n, 36] and the hidden activations."""
    P = unflatten(theta, hidden)
    h1 = np.maximum(F @ P["W1"].T + P["b1"], 0.0)
    h2 = np.maximum(h1 @ P["W2"].T + P["b2"], 0.0)
    h3 = np.maximum(h2 @ P["W3"].T + P["b3"], 0.0)
    o = h3 @ P["W4"].T + P["b4"]
    return o, (h1, h2, h3)


def split_outputs(o, F):
    """Per component: logits [n,4], normalised means [n,4,4], raw log-stds
    [n,4,4] (before clipping)."""
    o = np.asarray(o, dtype=np.float64).reshape(-1, NCOMP, 9)
    logit = o[:, :, 0]
    mean = o[:, :, 1:5].copy()
    mean[:, :, 0] += F[:, None, 0]
    mean[:, :, 2] += F[:, None, 1]
    return logit, mean, o[:, :, 5:9]


def log_softmax(a):
    mx = a.max(axis=-1, keepdims=True)
    return a - mx - np.log(np.exp(a - mx).sum(axis=-1, keepdims=True))


def mixture_table(p, Z, o):
    """Table of the births' proposal, 9 doubles per (measurement, component):
    log pi, mean (state units), standard deviation (state units)."""
    F = features(p, Z)
    logit, mean, s = split_outputs(o, F)
    O, S = scales(p)
    t = np.zeros((F.shape[0], NCOMP, 9))
    t[:, :, 0] = log_softmax(logit)
    t[:, :, 1:5] = O + S * mean
    t[:, :, 5:9] = S * np.exp(np.clip(s, LOGSTD_MIN, LOGSTD_MAX))
    return t


def nll_terms(p, o, F, X):
    """Per-pair loss and d loss / d o."""
    O, S = scales(p)
    xi = (np.asarray(X, dtype=np.float64).reshape(-1, 4) - O) / S
    logit, mean, sraw = split_outputs(o, F)
    s = np.clip(sraw, LOGSTD_MIN, LOGSTD_MAX)
    sig = np.exp(s)
    e = (xi[:, None, :] - mean) / sig                      # [n, c, d]
    logN = np.sum(-0.5 * e * e - s - 0.5 * LOG_2PI, axis=2)  # [n, c]
    logpi = log_softmax(logit)
    a = logpi + logN
    mx = a.max(axis=1, keepdims=True)
    lse = mx[:, 0] + np.log(np.exp(a - mx).sum(axis=1))
    loss = -lse
    r = np.exp(a - lse[:, None])                           # responsibilities
    pi = np.exp(logpi)
    g = np.zeros((F.shape[0], NCOMP, 9))
    g[:, :, 0] = pi - r
    g[:, :, 1:5] = -r[:, :, None] * e / sig
    inside = (sraw > LOGSTD_MIN) & (sraw < LOGSTD_MAX)
    g[:, :, 5:9] = -r[:, :, None] * (e * e - 1.0) * inside
    return loss, g.reshape(-1, NOUT)


def loss_and_grad(p, theta, Z, X, hidden=128):
    """Mean loss over the pairs and its gradient (flat, like theta)."""
    F = features(p, Z)
    n = F.shape[0]
    P = unflatten(theta, hidden)
    o, (h1, h2, h3) = forward(theta, F, hidden)
    loss, go = nll_terms(p, o, F, X)
    go = go / n
    G = {"W4": go.T @ h3, "b4": go.sum(axis=0)}
    d3 = (go @ P["W4"]) * (h3 > 0)
    G["W3"], G["b3"] = d3.T @ h2, d3.sum(axis=0)
    d2 = (d3 @ P["W3"]) * (h2 > 0)
    G["W2"], G["b2"] = d2.T @ h1, d2.sum(axis=0)
    d1 = (d2 @ P["W2"]) * (h1 > 0)
    G["W1"], G["b1"] = d1.T @ F, d1.sum(axis=0)
    return float(loss.mean()), flatten(G, hidden)


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba, 2015) at step number t >= 1."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
