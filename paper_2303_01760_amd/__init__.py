"""MI355X-native hybrid scattered-regular meshless stencils (build, apply, step)."""
