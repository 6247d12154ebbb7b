"""Seeded synthetic detectors and events shared by the oracle tests and the
GPU path.  Simulation only: no part of the track finder lives here."""
from .detector import Detector, barrel10, barrel_endcap  # noqa: F401
from .events import Event, make_event, make_batch, concat_events  # noqa: F401
