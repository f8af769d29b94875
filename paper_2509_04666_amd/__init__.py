"""MI355X-native known-object prediction hot path (n-body propagation,
universal-variable light-time hops, sky-binned field-of-view test)."""
__version__ = "0.1.0"
