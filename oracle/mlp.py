"""FP64 reference of the committor model and its training step (test
infrastructure only).

Model: phi_k = (log1p(x_k) - mean_k) * inv_std_k; h1 = tanh(W1 phi + b1);
h2 = tanh(W2 h1 + b2); z = W3 . h2 + b3; q = sigmoid(z).
Loss: mean over the batch of the binary cross-entropy with soft label y,
written as max(z,0) - z y + log(1 + e^{-|z|}).
Gradient: the chain rule written out layer by layer (dL/dz = (q - y)/B).
Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
Parameter order: W1[64][n_in], b1[64], W2[64][64], b2[64], W3[64], b3.
"""
import numpy as np

H = 64


def unpack(p, n_in):
    p = np.asarray(p, np.float64)
    o = 0
    W1 = p[o:o + H * n_in].reshape(H, n_in); o += H * n_in
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, W3, b3


def features(x, feat, n_in):
    feat = np.asarray(feat, np.float64)
    return (np.log1p(np.asarray(x, np.float64)) - feat[:n_in]) * feat[n_in:]


def forward(p, feat, x, n_in):
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in)
    phi = features(x, feat, n_in)
    h1 = np.tanh(phi @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    z = h2 @ W3 + b3
    return phi, h1, h2, z


def loss(p, feat, x, y, n_in):
    _, _, _, z = forward(p, feat, x, n_in)
    y = np.asarray(y, np.float64)
    return float(np.mean(np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def loss_grad(p, feat, x, y, n_in):
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in)
    phi, h1, h2, z = forward(p, feat, x, n_in)
    y = np.asarray(y, np.float64)
    B = len(y)
    q = 1.0 / (1.0 + np.exp(-z))
    g3 = (q - y) / B                          # dL/dz
    dW3 = g3 @ h2
    db3 = g3.sum()
    g2 = np.outer(g3, W3) * (1.0 - h2 ** 2)   # dL/d(pre-activation of layer 2)
    dW2 = g2.T @ h1
    db2 = g2.sum(axis=0)
    g1 = (g2 @ W2) * (1.0 - h1 ** 2)
    dW1 = g1.T @ phi
    db1 = g1.sum(axis=0)
    grad = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3, [db3]])
    return loss(p, feat, x, y, n_in), grad


def adam(p, m, v, g, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
