"""MI355X-native ternary flip-graph walks (libtsf): see include/tsf.h."""
