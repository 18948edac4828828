"""Learned warm start: the small convolutional network that proposes inverse-
depth and bias corrections for a window before Gauss-Newton, in FP64.

The paper has no counterpart of this network (its learned part is the
correspondence network that produces u* and w, Sec. 3.1); this module is the
reference definition the GPU kernels are checked against.  Everything here is
plain NumPy float64 written out from the definitions below.

Inputs per keyframe i (as the source of its outgoing edges), on a grid of
4 x 4-pixel cells (hq = ceil(H/4), wq = ceil(W/4)); every quantity of a cell
is taken over its full-resolution pixels and the valid pixel-residuals of
the keyframe's outgoing edges at the current state (Eq. 1):
  ch 0   sum w_x r_x / (sum w_x + 1e-6)          weighted mean x residual, px
  ch 1   sum w_y r_y / (sum w_y + 1e-6)          weighted mean y residual, px
  ch 2   sum (w_x + w_y) / (2 k n_cell)           mean confidence (k edges)
  ch 3   mean inverse depth of the cell
  ch 4-12  the inertial residual (Eq. 3) of the factor (i, i+1) at the current
         state, rotation x 100, position x 10, velocity x 10, as constant
         planes (zero for the last keyframe)
  ch 13  -sum(w_x J_dx r_x + w_y J_dy r_y) / (h + 1e-6) / 0.2, the cell's
         depth-only Gauss-Newton step (poses held) in units of 0.2, where
         J_d = dr/dd is the inverse-depth column of the Jacobian of Eq. 1 and
         h = sum(w_x J_dx^2 + w_y J_dy^2)
  ch 14  log(1 + h / n_cell), the depth information per pixel
Network (weights W, biases b, zero padding 1, ReLU after each of 4 layers):
  h1 = relu(conv3x3(x, 15 -> 32)), h2..h4 = relu(conv3x3(h, 32 -> 32))
  dd = conv3x3(h4, 32 -> 1)                      inverse-depth correction per cell
  db = Wb mean_cells(h4) + bb                    bias correction (6) of keyframe i
Cells outside a keyframe's grid (images of different sizes share one padded
canvas) are zero in every layer and excluded from the pooling and the loss.
The full-resolution correction is the bilinear upsampling of dd by 4 (cell
centres at 4 c + 1.5, clamped at the borders).
Loss (one batch of keyframes):
  L = mean_{img, valid cell} ((dd - dd*) / s_d)^2 + mean_img sum_6 ((db - db*) / s_b)^2
with s_d = 0.02 and s_b = (0.005 x 3, 0.05 x 3); the labels dd*, db* are the
converged plain Gauss-Newton solution minus the initial state (dd* averaged
over each cell).  Training uses AdamW (decoupled weight decay).

Test infrastructure (see the package header).  Pinned by: conv3x3 against
scipy.signal.correlate2d, the whole backward pass against central finite
differences, the AdamW step against its closed form for zero moments, the
upsampling against constant and linear inputs, zero residual channels on
noiseless ground truth, every input channel of a hand-built two-keyframe
window against values worked out from its geometry (unequal x / y weights,
a factor with known deltas), and the loss against its value on a two-image
example with a masked cell.
"""
import numpy as np

from . import imu as imu_mod
from . import vision

C_IN = 15
C = 32
N_LAYERS = 4
S_D = 0.02
S_B = np.array([0.005] * 3 + [0.05] * 3)
FEAT_SCALE_IMU = np.array([100.0] * 3 + [10.0] * 6)
FEAT_SCALE_STEP = 0.2

# flat parameter layout
SHAPES = [("W1", (C, C_IN, 3, 3)), ("b1", (C,)),
          ("W2", (C, C, 3, 3)), ("b2", (C,)),
          ("W3", (C, C, 3, 3)), ("b3", (C,)),
          ("W4", (C, C, 3, 3)), ("b4", (C,)),
          ("Wd", (1, C, 3, 3)), ("bd", (1,)),
          ("Wb", (6, C)), ("bb", (6,))]


def n_params():
    return int(sum(np.prod(s) for _, s in SHAPES))


def unpack(theta):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], np.float64).ravel() for name, _ in SHAPES])


def init_params(seed):
    """He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = {}
    for name, shp in SHAPES:
        if name.startswith("b"):
            parts[name] = np.zeros(shp)
        else:
            fan_in = int(np.prod(shp[1:]))
            parts[name] = rng.standard_normal(shp) * np.sqrt(2.0 / fan_in)
    return pack(parts)


# --------------------------------------------------------------------------
# layers
# --------------------------------------------------------------------------
def conv3x3(x, W, b):
    """y[n, o, r, c] = b[o] + sum_{i, dy, dx} W[o, i, dy, dx] x[n, i, r + dy - 1, c + dx - 1]
    with zero padding; x (B, Cin, h, w)."""
    B, Ci, h, w = x.shape
    Co = W.shape[0]
    xp = np.zeros((B, Ci, h + 2, w + 2))
    xp[:, :, 1:h + 1, 1:w + 1] = x
    y = np.zeros((B, Co, h, w)) + b[None, :, None, None]
    for dy in range(3):
        for dx in range(3):
            patch = xp[:, :, dy:dy + h, dx:dx + w]              # (B, Ci, h, w)
            y += np.einsum("oi,nirc->norc", W[:, :, dy, dx], patch)
    return y


def conv3x3_backward(x, W, gy):
    """Gradients of conv3x3 with respect to x, W and b for the output gradient gy."""
    B, Ci, h, w = x.shape
    xp = np.zeros((B, Ci, h + 2, w + 2))
    xp[:, :, 1:h + 1, 1:w + 1] = x
    gxp = np.zeros_like(xp)
    gW = np.zeros_like(W)
    for dy in range(3):
        for dx in range(3):
            patch = xp[:, :, dy:dy + h, dx:dx + w]
            gW[:, :, dy, dx] = np.einsum("norc,nirc->oi", gy, patch)
            gxp[:, :, dy:dy + h, dx:dx + w] += np.einsum("oi,norc->nirc", W[:, :, dy, dx], gy)
    gb = gy.sum(axis=(0, 2, 3))
    return gxp[:, :, 1:h + 1, 1:w + 1], gW, gb


def forward(theta, x, mask):
    """x (B, 15, h, w) on the padded canvas, mask (B, h, w) of valid cells.
    Returns dd (B, h, w), db (B, 6) and the activations for the backward pass."""
    P = unpack(theta)
    m = mask[:, None].astype(np.float64)
    acts = [x * m]
    h = acts[0]
    for l in range(1, N_LAYERS + 1):
        h = np.maximum(conv3x3(h, P[f"W{l}"], P[f"b{l}"]), 0.0) * m
        acts.append(h)
    dd = conv3x3(h, P["Wd"], P["bd"])[:, 0] * mask
    cnt = np.maximum(mask.sum(axis=(1, 2)), 1.0)
    pooled = h.sum(axis=(2, 3)) / cnt[:, None]
    db = pooled @ P["Wb"].T + P["bb"][None]
    return dd, db, (acts, pooled, cnt)


def loss(dd, db, dd_lab, db_lab, mask):
    nv = max(float(mask.sum()), 1.0)
    ed = (dd - dd_lab) / S_D * mask
    eb = (db - db_lab) / S_B[None]
    B = db.shape[0]
    return float((ed ** 2).sum() / nv + (eb ** 2).sum() / B)


def backward(theta, x, mask, dd_lab, db_lab):
    """Loss and its gradient with respect to theta (flat)."""
    P = unpack(theta)
    dd, db, (acts, pooled, cnt) = forward(theta, x, mask)
    L = loss(dd, db, dd_lab, db_lab, mask)
    nv = max(float(mask.sum()), 1.0)
    B = db.shape[0]
    g_dd = 2.0 * (dd - dd_lab) / S_D ** 2 * mask / nv
    g_db = 2.0 * (db - db_lab) / S_B[None] ** 2 / B
    grads = {}
    grads["Wb"] = g_db.T @ pooled
    grads["bb"] = g_db.sum(axis=0)
    g_pooled = g_db @ P["Wb"]
    h4 = acts[N_LAYERS]
    m = mask[:, None].astype(np.float64)
    gh, grads["Wd"], grads["bd"] = conv3x3_backward(h4, P["Wd"], g_dd[:, None])
    gh = gh + (g_pooled / cnt[:, None])[:, :, None, None] * m
    for l in range(N_LAYERS, 0, -1):
        gpre = gh * (acts[l] > 0) * m
        gx, grads[f"W{l}"], grads[f"b{l}"] = conv3x3_backward(acts[l - 1], P[f"W{l}"], gpre)
        gh = gx * m
    return L, pack(grads)


def adamw_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8, wd=1e-4):
    """One AdamW step (t = 1, 2, ...): moments, bias correction, decoupled decay."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    theta = theta - lr * (mh / (np.sqrt(vh) + eps) + wd * theta)
    return theta, m, v


def upsample4(dd_cells, H, W):
    """Bilinear upsampling of a (hq, wq) cell grid to (H, W): pixel (y, x) reads
    the grid at ((y - 1.5) / 4, (x - 1.5) / 4), clamped to the grid."""
    hq, wq = dd_cells.shape
    out = np.zeros((H, W))
    for y in range(H):
        fy = min(max((y - 1.5) / 4.0, 0.0), hq - 1.0)
        y0 = int(np.floor(fy))
        y1 = min(y0 + 1, hq - 1)
        ay = fy - y0
        for x in range(W):
            fx = min(max((x - 1.5) / 4.0, 0.0), wq - 1.0)
            x0 = int(np.floor(fx))
            x1 = min(x0 + 1, wq - 1)
            ax = fx - x0
            out[y, x] = ((1 - ay) * ((1 - ax) * dd_cells[y0, x0] + ax * dd_cells[y0, x1])
                         + ay * ((1 - ax) * dd_cells[y1, x0] + ax * dd_cells[y1, x1]))
    return out


# --------------------------------------------------------------------------
# input features of one window
# --------------------------------------------------------------------------
def features(cam, state, graph, z_min=0.1, hq=None, wq=None, use_imu=True):
    """(N, 15, hq, wq) features and (N, hq, wq) validity of the cells of each
    keyframe, following the channel list in the module header."""
    fx, fy, cx, cy, H, W = cam.intr
    N = state.R.shape[0]
    hq0, wq0 = (H + 3) // 4, (W + 3) // 4
    hq = hq0 if hq is None else hq
    wq = wq0 if wq is None else wq
    X = np.zeros((N, C_IN, hq, wq))
    mask = np.zeros((N, hq, wq))
    mask[:, :hq0, :wq0] = 1.0
    ys, xs = np.mgrid[0:H, 0:W]
    cell = (ys // 4) * wq0 + (xs // 4)
    ncell = np.bincount(cell.ravel(), minlength=hq0 * wq0).astype(np.float64)
    for i in range(N):
        sxr = np.zeros(hq0 * wq0)
        syr = np.zeros(hq0 * wq0)
        swx = np.zeros(hq0 * wq0)
        swy = np.zeros(hq0 * wq0)
        sg = np.zeros(hq0 * wq0)
        sh = np.zeros(hq0 * wq0)
        k = 0
        for e in range(len(graph.ii)):
            if int(graph.ii[e]) != i:
                continue
            j = int(graph.jj[e])
            k += 1
            r, valid, _, J_d = vision.edge_linearize_body(cam.intr, cam.T_bc, state.R[i], state.p[i], state.R[j],
                                                          state.p[j], state.d[i], graph.target[e], z_min)
            w = np.asarray(graph.weight[e], np.float64).reshape(2, -1) * valid[None]
            c = cell.ravel()
            sg += np.bincount(c, weights=w[0] * J_d[0] * r[0] + w[1] * J_d[1] * r[1], minlength=hq0 * wq0)
            sh += np.bincount(c, weights=w[0] * J_d[0] ** 2 + w[1] * J_d[1] ** 2, minlength=hq0 * wq0)
            sxr += np.bincount(c, weights=w[0] * r[0], minlength=hq0 * wq0)
            syr += np.bincount(c, weights=w[1] * r[1], minlength=hq0 * wq0)
            swx += np.bincount(c, weights=w[0], minlength=hq0 * wq0)
            swy += np.bincount(c, weights=w[1], minlength=hq0 * wq0)
        X[i, 0, :hq0, :wq0] = (sxr / (swx + 1e-6)).reshape(hq0, wq0)
        X[i, 1, :hq0, :wq0] = (syr / (swy + 1e-6)).reshape(hq0, wq0)
        X[i, 2, :hq0, :wq0] = ((swx + swy) / (2.0 * max(k, 1) * ncell)).reshape(hq0, wq0)
        dsum = np.bincount(cell.ravel(), weights=np.asarray(state.d[i], np.float64).ravel(), minlength=hq0 * wq0)
        X[i, 3, :hq0, :wq0] = (dsum / ncell).reshape(hq0, wq0)
        X[i, 13, :hq0, :wq0] = (-sg / (sh + 1e-6) / FEAT_SCALE_STEP).reshape(hq0, wq0)
        X[i, 14, :hq0, :wq0] = np.log1p(sh / ncell).reshape(hq0, wq0)
        if use_imu and i + 1 < N:
            P = graph.factors[i]
            r = imu_mod.residual(state.R[i], state.p[i], state.v[i], state.b[i],
                                 state.R[i + 1], state.p[i + 1], state.v[i + 1], state.b[i + 1], P, cam.gravity)
            X[i, 4:13, :hq0, :wq0] = (r[:9] * FEAT_SCALE_IMU)[:, None, None]
    return X, mask


def cell_mean(a, H, W):
    """Mean of a full-resolution map (H, W) over each 4 x 4 cell."""
    hq0, wq0 = (H + 3) // 4, (W + 3) // 4
    ys, xs = np.mgrid[0:H, 0:W]
    cell = ((ys // 4) * wq0 + (xs // 4)).ravel()
    s = np.bincount(cell, weights=np.asarray(a, np.float64).ravel(), minlength=hq0 * wq0)
    n = np.bincount(cell, minlength=hq0 * wq0)
    return (s / n).reshape(hq0, wq0)
