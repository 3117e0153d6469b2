"""MI355X-native planar Quickhull (placeholder; the binding is filled in next)."""
