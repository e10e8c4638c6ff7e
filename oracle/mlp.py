"""FP64 reference of the selector MLP (test infrastructure only): forward pass, class-
weighted softmax cross-entropy and its gradient by plain backpropagation, and one Adam
step, written with numpy.  Parameter layout as in the library: W1 16x64 at 0, b1 at
1024, W2 64x64 at 1088, b2 at 5184, W3 64x8 at 5248, b3 at 5760 (row-major [in][out])."""
import numpy as np

NF, NH, NC = 16, 64, 8
OFF = dict(W1=0, b1=1024, W2=1088, b2=5184, W3=5248, b3=5760)
NPARAM = 5768


def unpack(w):
    w = np.asarray(w, np.float64)
    return (w[0:1024].reshape(NF, NH), w[1024:1088], w[1088:5184].reshape(NH, NH), w[5184:5248],
            w[5248:5760].reshape(NH, NC), w[5760:5768])


def forward(w, X, mu, isd):
    W1, b1, W2, b2, W3, b3 = unpack(w)
    Xn = (np.asarray(X, np.float64) - mu) * isd
    H1 = np.maximum(Xn @ W1 + b1, 0.0)
    H2 = np.maximum(H1 @ W2 + b2, 0.0)
    return Xn, H1, H2, H2 @ W3 + b3


def loss_and_grad(w, X, y, cw, mu, isd):
    W1, b1, W2, b2, W3, b3 = unpack(w)
    Xn, H1, H2, Z = forward(w, X, mu, isd)
    Z = Z - Z.max(1, keepdims=True)
    P = np.exp(Z)
    P /= P.sum(1, keepdims=True)
    wt = np.asarray(cw, np.float64)[y]
    wt = wt / wt.sum()
    loss = float(-(wt * np.log(P[np.arange(len(y)), y])).sum())
    dZ = P.copy()
    dZ[np.arange(len(y)), y] -= 1.0
    dZ *= wt[:, None]
    dH2 = (dZ @ W3.T) * (H2 > 0)
    dH1 = (dH2 @ W2.T) * (H1 > 0)
    g = np.concatenate([(Xn.T @ dH1).ravel(), dH1.sum(0), (H1.T @ dH2).ravel(), dH2.sum(0), (H2.T @ dZ).ravel(),
                        dZ.sum(0)])
    return loss, g


def adam(w, g, m, v, step, lr, b1, b2, eps, wd):
    g = g + wd * w
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16(x):
    """Round to BF16 (nearest even) and back, as the library's inference does."""
    a = np.asarray(x, np.float32).copy()
    u = a.view(np.uint32)
    u += 0x7FFF + ((u >> 16) & 1)
    u &= 0xFFFF0000
    return a.astype(np.float64)


def forward_bf16(w, X, mu, isd):
    """Logits with weights, normalised inputs and hidden activations rounded to BF16,
    FP32-like accumulation (computed here in FP64)."""
    W1, b1, W2, b2, W3, b3 = unpack(w)
    Xn = bf16((np.asarray(X, np.float32) - np.float32(mu)) * np.float32(isd))
    H1 = bf16(np.maximum(Xn @ bf16(W1) + b1, 0.0))
    H2 = bf16(np.maximum(H1 @ bf16(W2) + b2, 0.0))
    return H2 @ bf16(W3) + b3
