"""MI355X-native whole-population GP fitness evaluation (TensorGP's hot path)."""
