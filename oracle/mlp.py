"""Reference forward/backward of the near-field surrogate network (FP64).

Architecture: x (16) -> tanh(x W1 + b1) (128) -> tanh(. W2 + b2) (128)
-> tanh(. W3 + b3) (128) -> . W4 + b4 (6); loss = mean over the batch and the
six outputs of (y - t)^2.  Weights are row-major [in][out].  The flat
parameter layout (W1, b1, W2, b2, W3, b3, W4, b4) is the one the GPU library
exchanges through fagbi_mlp_get_weights / fagbi_mlp_set_weights.

Parity unpinned by the paper (it has no learned part); pinned here by finite
differences of the loss (tests/test_mlp_oracle.py).
"""
import numpy as np

SIZES = [(16, 128), (128, 128), (128, 128), (128, 6)]


def n_params():
    return sum(a * b + b for a, b in SIZES)


def unpack(theta):
    theta = np.asarray(theta, np.float64)
    out, k = [], 0
    for a, b in SIZES:
        W = theta[k:k + a * b].reshape(a, b)
        k += a * b
        bb = theta[k:k + b]
        k += b
        out.append((W, bb))
    return out


def forward(theta, X):
    layers = unpack(theta)
    hs = [np.asarray(X, np.float64)]
    for li, (W, b) in enumerate(layers):
        z = hs[-1] @ W + b
        hs.append(np.tanh(z) if li < len(layers) - 1 else z)
    return hs


def loss_and_grad(theta, X, T):
    """mean squared error and its gradient w.r.t. the flat parameters"""
    layers = unpack(theta)
    hs = forward(theta, X)
    Y = hs[-1]
    n = Y.size
    loss = float(((Y - T) ** 2).sum() / n)
    d = 2.0 * (Y - T) / n
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        gW = hs[li].T @ d
        gb = d.sum(0)
        grads.append((gW, gb))
        if li > 0:
            d = (d @ W.T) * (1.0 - hs[li] ** 2)
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat
