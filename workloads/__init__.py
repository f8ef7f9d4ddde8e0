"""Seeded synthetic inputs shared by the tests, the benchmark and the server
demo.  Holds no point-in-polygon arithmetic: it only draws points and
polygons (see ``gen.py``)."""
from .gen import *  # noqa: F401,F403
