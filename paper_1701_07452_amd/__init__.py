"""MI355X-native per-patch ideal-MHD update (MHDTVD + CTU + constrained transport)."""
