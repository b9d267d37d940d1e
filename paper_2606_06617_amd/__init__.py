"""MI355X-native PSWF-LR reciprocal-space path (package root)."""
