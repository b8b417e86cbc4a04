"""Pose comparison shared by the tracker tests."""
import numpy as np


def pose_error(A, B):
    """(translation error in m, rotation angle in degrees) between two
    world->camera poses, compared as camera->world transforms"""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    Ra, Rb = A[:3, :3].T, B[:3, :3].T
    ta, tb = -(Ra @ A[:3, 3]), -(Rb @ B[:3, 3])
    dR = Ra @ Rb.T
    w = np.array([dR[2, 1] - dR[1, 2], dR[0, 2] - dR[2, 0], dR[1, 0] - dR[0, 1]]) / 2
    return float(np.linalg.norm(ta - tb)), float(np.degrees(np.arcsin(min(1.0, np.linalg.norm(w)))))
