"""MI355X-native FFT phase-field-fracture toughness homogenization."""
