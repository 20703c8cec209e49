"""MI355X-native hot path of the unified gas-kinetic wave-particle (UGKWP) method."""
