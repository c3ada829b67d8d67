"""MI355X-native discord search (PhiDD / HOTSAX hot path) behind a C ABI.

The compute path lives in the HIP library ``lib/libdiscord.so`` built from
``csrc/``; this package only marshals arguments to it.  Importing the package
does not load the library; the first call that needs it does, and raises if it
is missing (there is no CPU fallback).
"""
from ._binding import *  # noqa: F401,F403
