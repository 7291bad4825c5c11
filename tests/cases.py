"""Hand-built inputs shared by the CPU pins and the GPU parity tests (no
arithmetic of the method here: only matrices, vectors and network weights
written down from their definitions)."""
import numpy as np


def two_cell_blocks(A6):
    """(2, 7, 3, 3) stencil blocks of a 2x1x1 grid holding the 6x6 matrix A6
    (slots -z,-y,-x,D,+x,+y,+z; cell 0 couples to cell 1 through +x)."""
    B = np.zeros((2, 7, 3, 3))
    B[0, 3], B[0, 4] = A6[0:3, 0:3], A6[0:3, 3:6]
    B[1, 2], B[1, 3] = A6[3:6, 0:3], A6[3:6, 3:6]
    return B


def skew6():
    """An invertible skew-symmetric 6x6 matrix with dyadic entries (all the
    products and sums BiCGSTAB forms on it below are exact in FP64)."""
    K = np.zeros((6, 6))
    for i, j, v in ((0, 1, -0.75), (1, 2, 0.5), (2, 5, 0.5), (3, 4, 0.25), (1, 4, 1.0), (2, 3, -0.5),
                    (4, 5, 2.0)):
        K[i, j], K[j, i] = v, -v
    return K


def breakdown_systems():
    """(name, matrix, b, x BiCGSTAB hands back) for its two breakdown exits,
    unpreconditioned, from x0 = 0:
      rv0    -- A skew-symmetric, so r^ . A r^ = 0 in the first iteration
                (alpha undefined); x stays 0;
      omega0 -- A = e0 e0^T + K and b = (1,1,1,1,0,0): rho = |b|^2 = 4,
                r^ . A b = b_0^2 = 1, alpha = 4, s = b - 4 A b has s_0 = 0, so
                t . s = s^T A s = s_0^2 = 0 and omega = 0; x = alpha b."""
    K = skew6()
    P = np.zeros((6, 6))
    P[0, 0] = 1.0
    b_skew = np.array([1.0, 2.0, -1.0, 3.0, 1.0, -2.0])
    b_om = np.array([1.0, 1.0, 1.0, 1.0, 0.0, 0.0])
    return [("rv0", K, b_skew, np.zeros(6)), ("omega0", P + K, b_om, 4.0 * b_om)]


def unet_layout(c0=16, c1=32, c2=64):
    """(offset, weight count, cout, fan-in) per layer of the U-Net parameter
    vector: layers 0..9 are 3x3x3 convs stored w[tap][ci][co] then b[co],
    layer 10 the final 1x1x1 layer w[ci][co] then b."""
    cin = [4, c0, c0, c1, c1, c2, c2, c1, c1, c0, c0]
    cout = [c0, c0, c1, c1, c2, c2, c1, c1, c0, c0, 3]
    out, off = [], 0
    for l in range(11):
        nw = (27 if l < 10 else 1) * cin[l] * cout[l]
        out.append((off, nw, cout[l], cin[l] * (27 if l < 10 else 1)))
        off += nw + cout[l]
    return out, off


def identity_unet(c0=16, c1=32, c2=64):
    """Weights (all 0 or +-1, exact in BF16) under which the network maps its
    three residual channels to themselves: the first conv's centre tap sends
    channel p to +x_p and -x_p, whose ReLUs relu(x) - relu(-x) = x pass the
    second conv's and the last level-1 conv's centre-tap identities and the
    additive skip (every deeper layer is zero), and the final 1x1x1 layer
    forms the difference.  The preconditioner z = s N(v/s) is then the
    identity up to the BF16 rounding of v/s."""
    lay, n = unet_layout(c0, c1, c2)
    p = np.zeros(n)
    centre = 13
    off = lay[0][0]
    for q in range(3):
        p[off + (centre * 4 + q) * c0 + 2 * q] = 1.0
        p[off + (centre * 4 + q) * c0 + 2 * q + 1] = -1.0
    for l in (1, 9):
        off = lay[l][0]
        for c in range(6):
            p[off + (centre * c0 + c) * c0 + c] = 1.0
    off = lay[10][0]
    for q in range(3):
        p[off + (2 * q) * 3 + q] = 1.0
        p[off + (2 * q + 1) * 3 + q] = -1.0
    return p
