"""Seeded synthetic inputs for photometric bundle adjustment.

This package only produces input data (images, poses, points, observation
lists). It contains none of the solver's arithmetic; the CPU oracle and the
GPU library both consume its arrays.
"""
from .configs import BUILDERS, HUBER_K, PATTERN8, Scene, learned, mid, precision, tiny, window

__all__ = ["BUILDERS", "HUBER_K", "PATTERN8", "Scene", "tiny", "mid", "precision", "learned", "window"]
