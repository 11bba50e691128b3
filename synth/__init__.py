"""Seeded synthetic UT events: the only module that both the oracle's tests and the HIP path's tests use.

It simulates the detector (geometry, a single-kick field model, hit smearing, noise, raw-bank
encoding) and holds none of the reconstruction method's arithmetic: no decoding, no window search,
no tracklet finding, no fit.  Random numbers come from ``numpy.random.default_rng(seed)`` (PCG64),
so every consumer sees the same bytes for the same (config, seed).
"""
from .detector import Detector, make_detector, CompassParams, make_compass_params
from .events import EventBatch, generate, take_events, CONFIGS, config

__all__ = ["Detector", "make_detector", "CompassParams", "make_compass_params",
           "EventBatch", "generate", "take_events", "CONFIGS", "config"]
