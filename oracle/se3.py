"""SE(3) helpers in float64 for the prediction step and the pose read-out.

Sec. III-A (prediction step): each particle moves as x_t = x_{t-1} * O_t * x_eps
with x_eps = Exp(delta) the exponential map of a Gaussian twist delta in se(3).
Poses are 3x4 camera-to-world matrices [R | t].  A twist is (rho, phi):
translation part rho, rotation part phi.
"""
import numpy as np


def hat(v):
    """The 3x3 skew matrix of v: hat(v) @ w == cross(v, w)."""
    x, y, z = v
    return np.array([[0.0, -z, y], [z, 0.0, -x], [-y, x, 0.0]])


def exp_se3(rho, phi):
    """SE(3) exponential of the twist (rho, phi), as a 3x4 [R | t].

    R = I + a K + b K^2 and t = (I + b K + c K^2) rho with K = hat(phi),
    theta = |phi|, a = sin(theta)/theta, b = (1 - cos(theta))/theta^2,
    c = (theta - sin(theta))/theta^3 (Rodrigues' formula and the left Jacobian);
    near theta = 0 the coefficients take their Taylor series."""
    rho = np.asarray(rho, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    th2 = float(phi @ phi)
    th = np.sqrt(th2)
    K = hat(phi)
    K2 = K @ K
    if th < 1e-4:
        a = 1.0 - th2 / 6.0 + th2 * th2 / 120.0
        b = 0.5 - th2 / 24.0 + th2 * th2 / 720.0
        c = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0
    else:
        a = np.sin(th) / th
        b = (1.0 - np.cos(th)) / th2
        c = (th - np.sin(th)) / (th2 * th)
    R = np.eye(3) + a * K + b * K2
    V = np.eye(3) + b * K + c * K2
    out = np.zeros((3, 4))
    out[:, :3] = R
    out[:, 3] = V @ rho
    return out


def compose(A, B):
    """A * B for 3x4 rigid transforms."""
    out = np.zeros((3, 4))
    out[:, :3] = A[:, :3] @ B[:, :3]
    out[:, 3] = A[:, :3] @ B[:, 3] + A[:, 3]
    return out


def to4(P):
    M = np.eye(4)
    M[:3, :] = P
    return M


def pose_estimate(poses, w):
    """Read a pose out of a weighted particle set (the paper does not say how):
    weighted mean position, and the chordal L2 mean rotation, i.e. the rotation
    nearest in Frobenius norm to sum_i w_i R_i: U diag(1, 1, det(U V^T)) V^T from
    the SVD U S V^T of that sum."""
    poses = np.asarray(poses, dtype=np.float64).reshape(-1, 3, 4)
    w = np.asarray(w, dtype=np.float64)
    w = w / w.sum()
    t = (w[:, None] * poses[:, :, 3]).sum(0)
    M = (w[:, None, None] * poses[:, :, :3]).sum(0)
    U, _, Vt = np.linalg.svd(M)
    D = np.diag([1.0, 1.0, np.sign(np.linalg.det(U @ Vt))])
    out = np.zeros((3, 4))
    out[:, :3] = U @ D @ Vt
    out[:, 3] = t
    return out


def rotation_angle_deg(Ra, Rb):
    """Angle of Ra^T Rb in degrees, atan2(|vee(skew part)|, (trace - 1) / 2)."""
    M = Ra.T @ Rb
    s = 0.5 * np.array([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]])
    c = 0.5 * (np.trace(M) - 1.0)
    return float(np.degrees(np.arctan2(np.linalg.norm(s), c)))


def pose_errors(P_est, P_ref):
    """(position error in scene units, rotation error in degrees)."""
    return (float(np.linalg.norm(P_est[:, 3] - P_ref[:, 3])),
            rotation_angle_deg(P_est[:, :3], P_ref[:, :3]))
